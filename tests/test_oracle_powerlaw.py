"""Pins of the oracle's power-law local relaxation time (Sec. 5, Eqs. nn1-nn7)."""
import numpy as np
import pytest

import closed_forms as cf
from oracle import Oracle, OracleParams
from oracle.oracle import WALL

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OMEGA = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def feq(rho, ux, uy):
    eu = EX * ux + EY * uy
    return OMEGA * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))


def relaxed_tau(n, xi, tmin, tmax, a, b, rho=1.02, ux=0.01, uy=-0.02):
    """Uniform periodic state f = feq + f_neq with a prescribed traceless
    non-equilibrium stress [[a, b], [b, -a]]; after one step (streaming leaves a
    uniform state unchanged) f_neq has been scaled by 1 - 1/tau*."""
    Pi = np.array([[a, b], [b, -a]])
    e = np.stack([EX, EY], 1).astype(float)
    Q = np.einsum("ia,ib->iab", e, e) - np.eye(2) / 3
    fneq = 4.5 * OMEGA * np.einsum("iab,ab->i", Q, Pi)
    f = feq(rho, ux, uy) + fneq
    o = Oracle(OracleParams(nx=3, ny=3, tau=1.0, power_law=True, n_index=n, K=xi,
                            tau_min=tmin, tau_max=tmax))
    o.set_populations(np.broadcast_to(f[:, None, None], (9, 3, 3)).copy())
    o.run(1)
    f1 = o.populations()[:, 1, 1]
    ratio = np.dot(f1 - feq(rho, ux, uy), fneq) / np.dot(fneq, fneq)
    return 1.0 / (1.0 - ratio), Pi, rho


@pytest.mark.parametrize("n", [0.5, 0.75, 1.5, 2.0])
@pytest.mark.parametrize("xi", [1e-3, 1e-2])
def test_local_tau_satisfies_paper_relation(n, xi):
    """nu* = kappa |Pi_D|^((n-1)/2) xi with kappa = 2^(n-1) (Eq. nn4), where
    Pi_D = (1/4)(u_y + v_x)^2 - u_x v_y (Eq. nn3) of the strain rate
    D = -Pi_neq / (2 rho c_s^2 tau*), and tau* = 1/2 + 3 nu*, or the clamp."""
    tmin, tmax = 0.5001, 50.0
    hits = 0
    # tau* is read back from f_neq(t=1) / f_neq(t=0); rounding of f ~ 0.1 limits
    # that to ~1e-17 / |f_neq| relative, so the amplitudes stay >= 1e-7
    for amp in np.logspace(-7, -1, 13):
        for (a, b) in ((amp, 0.3 * amp), (-0.2 * amp, amp)):
            tau, Pi, rho = relaxed_tau(n, xi, tmin, tmax, a, b)
            D = -Pi / (2 * rho * tau / 3)
            PiD = D[0, 1] ** 2 - D[0, 0] * D[1, 1]
            nu = 2 ** (n - 1) * abs(PiD) ** ((n - 1) / 2) * xi
            t_expect = 0.5 + 3 * nu
            if tmin < t_expect < tmax:
                hits += 1
                assert abs(tau - t_expect) < 1e-6 * tau, (amp, tau, t_expect)
            else:
                assert abs(tau - (tmin if t_expect <= tmin else tmax)) < 1e-6 * tau
    assert hits >= 3


@pytest.mark.parametrize("n", [0.5, 1.5])
def test_fluid_at_rest_stays_at_rest(n):
    """Zero strain (gamma_dot = 0, where xi gamma_dot^(n-1) is 0 or infinite)
    takes a clamp bound and leaves the rest state exactly unchanged."""
    o = Oracle(OracleParams(nx=6, ny=5, tau=1.0, power_law=True, n_index=n, K=0.01))
    f0 = o.populations()
    o.run(10)
    assert np.abs(o.populations() - f0).max() < 1e-15


@pytest.mark.parametrize("n,tau_expect", [(0.5, 2.5), (1.5, 0.51)])
def test_weak_shear_relaxes_at_the_clamp_bound(n, tau_expect):
    """A shear wave of amplitude 1e-7 has gamma_dot ~ 5e-9, far outside the
    unclamped range: it decays like the Newtonian wave at tau_max for n < 1 and
    at tau_min for n > 1, i.e. at nu k^2 up to the lattice correction, which
    grows as tau approaches 1/2."""
    ny, T, u0 = 128, 2000, 1e-7
    k = 2 * np.pi / ny
    y = np.arange(ny)
    ux = np.tile((u0 * np.sin(k * y))[:, None], (1, 4))

    def rate(**kw):
        o = Oracle(OracleParams(nx=4, ny=ny, **kw), ux=ux).run(T)
        u = o.moments()[1][:, 0]
        return np.log(u0 / ((u * np.sin(k * y)).sum() * 2 / ny)) / T
    r_pl = rate(tau=1.0, power_law=True, n_index=n, K=0.01, tau_min=0.51, tau_max=2.5)
    r_nw = rate(tau=tau_expect)
    assert abs(r_pl / r_nw - 1) < 1e-6
    assert abs(r_pl / (cf.nu_of_tau(tau_expect) * k * k) - 1) < 2e-2


def test_n_equal_one_is_newtonian_poiseuille():
    ny, g, K = 64, 1e-6, 0.1  # tau* = 1/2 + 3K = 0.8
    nu = K
    steps = int(27 * (ny - 2) ** 2 / (np.pi ** 2 * nu))
    o = Oracle(OracleParams(nx=4, ny=ny, bc_y=WALL, tau=1.0, gx=g, power_law=True,
                            n_index=1.0, K=K)).run(steps)
    ref = cf.poiseuille_exact(ny, 0.8, g)
    assert np.abs(o.moments()[1][1:-1, 0] - ref).max() / ref.max() < 5e-11


@pytest.mark.parametrize("n,g,steps,tol", [(0.5, 1.66e-5, 80000, 2e-3),
                                           (0.75, 3e-6, 220000, 6e-4)])
def test_clamped_powerlaw_channel(n, g, steps, tol):
    """Steady power-law channel (W = 64, K = 0.01, tau* in [0.51, 2.5]) against
    the closed form with the clamp; unclamped it is Eqs. nn6-nn7."""
    ny = 66
    o = Oracle(OracleParams(nx=4, ny=ny, bc_y=WALL, tau=1.0, gx=g, power_law=True, n_index=n,
                            K=0.01, tau_min=0.51, tau_max=2.5)).run(steps)
    u = o.moments()[1][1:-1, 0]
    ref = cf.powerlaw_channel(ny, n, 0.01, g, 0.51, 2.5)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < tol
    if n == 0.5:  # the clamp is active: the plain nn6-nn7 profile is further off
        unc = cf.powerlaw_channel_unclamped(ny, n, 0.01, g)
        assert np.linalg.norm(u - unc) / np.linalg.norm(unc) > 2 * tol


def test_shear_thickening_at_low_shear_is_fully_clamped():
    """n = 1.5, K = 0.01: xi gd^0.5 >= nu(0.51) = 1/300 needs gd >= 0.11, out of
    reach at low Mach, so every node relaxes with tau_min and the run equals the
    Newtonian run with tau = 0.51 bit for bit."""
    kw = dict(nx=4, ny=34, bc_y=WALL, gx=2.067e-8)
    a = Oracle(OracleParams(tau=1.0, power_law=True, n_index=1.5, K=0.01, tau_min=0.51,
                            tau_max=2.5, **kw)).run(2000)
    b = Oracle(OracleParams(tau=0.51, **kw)).run(2000)
    assert np.array_equal(a.populations(), b.populations())
