"""Pins of the oracle's BGK core (Sec. 2): collision, velocity-shift body force,
streaming, periodic wrap and halfway bounce-back, against closed forms and
exact invariants."""
import numpy as np
import pytest

import closed_forms as cf
from oracle import Oracle, OracleParams
from oracle.oracle import WALL

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


@pytest.mark.parametrize("tau", [0.7, 0.8, 1.0])
def test_poiseuille_exact_steady(tau):
    ny, g = 64, 1e-6
    nu = cf.nu_of_tau(tau)
    W = ny - 2
    steps = int(27 * W * W / (np.pi ** 2 * nu))
    o = Oracle(OracleParams(nx=4, ny=ny, bc_y=WALL, tau=tau, gx=g)).run(steps)
    rho, ux, uy = o.moments()
    ref = cf.poiseuille_exact(ny, tau, g)
    assert np.abs(ux[1:-1, :] - ref[:, None]).max() / ref.max() < 5e-11
    assert np.abs(uy).max() < 1e-10 * ref.max()


def test_channel_startup_at_5000_steps():
    """128x64 channel, walls y = 0 and 63, periodic x, g = 1e-6, tau = 0.8,
    5000 steps from rest: the flow is still developing, so the check is the
    start-up series (the steady parabola is reached only after ~1e5 steps)."""
    ny, nx, tau, g = 64, 128, 0.8, 1e-6
    o = Oracle(OracleParams(nx=nx, ny=ny, bc_y=WALL, tau=tau, gx=g)).run(5000)
    rho, ux, uy = o.moments()
    ref = cf.poiseuille_startup(ny, tau, g, 5000)
    d = ux[1:-1, :] - ref[:, None]
    assert np.sqrt((d ** 2).mean() / (ref ** 2).mean()) < 3e-4
    assert np.abs(ux - ux[:, :1]).max() < 1e-17  # x-invariance
    assert abs(o.mass() / (nx * (ny - 2)) - 1) < 1e-12


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_decay_rate(tau):
    """u_x = u0 sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3 (Sec. 2)."""
    ny, T, u0 = 128, 2000, 1e-4
    k = 2 * np.pi / ny
    y = np.arange(ny)
    ux = np.tile((u0 * np.sin(k * y))[:, None], (1, 8))
    o = Oracle(OracleParams(nx=8, ny=ny, tau=tau), ux=ux).run(T)
    _, u, v = o.moments()
    amp = (u[:, 0] * np.sin(k * y)).sum() * 2 / ny
    rate = np.log(u0 / amp) / T
    assert abs(rate / (cf.nu_of_tau(tau) * k * k) - 1) < 3e-3
    assert np.abs(v).max() < 1e-9 * u0


def test_mass_invariant_with_walls_and_obstacles():
    rng = np.random.default_rng(3)
    nx, ny = 40, 30
    mask = (rng.random((ny, nx)) < 0.15).astype(np.uint8)
    rho = 1 + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.02 * rng.standard_normal((ny, nx))
    uy = 0.02 * rng.standard_normal((ny, nx))
    o = Oracle(OracleParams(nx=nx, ny=ny, bc_y=WALL, tau=0.9, gx=1e-5, gy=-2e-5), mask,
               rho=rho, ux=ux, uy=uy)
    m0 = o.mass()
    o.run(300)
    assert abs(o.mass() - m0) / m0 < 1e-13


def test_momentum_gain_equals_body_force_periodic():
    """In a fully periodic domain collision adds rho g per node (the velocity
    shift of Sec. 2) and streaming conserves momentum: J(t+1) - J(t) = g M."""
    rng = np.random.default_rng(4)
    nx, ny, g = 24, 20, (3e-5, -1e-5)
    rho = 1 + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.03 * rng.standard_normal((ny, nx))
    uy = 0.03 * rng.standard_normal((ny, nx))
    o = Oracle(OracleParams(nx=nx, ny=ny, tau=0.75, gx=g[0], gy=g[1]), rho=rho, ux=ux, uy=uy)
    M = o.mass()
    for _ in range(5):
        j0 = np.array(o.momentum())
        o.run(1)
        j1 = np.array(o.momentum())
        np.testing.assert_allclose(j1 - j0, np.array(g) * M, rtol=1e-9, atol=1e-15)


def test_periodic_streaming_is_a_roll():
    """At tau = 1 and g = 0 collision returns feq(rho, j/rho); periodic
    streaming is then a cyclic shift of each plane by e_i."""
    rng = np.random.default_rng(6)
    nx, ny = 7, 5
    rho = 1 + 0.02 * rng.standard_normal((ny, nx))
    ux = 0.04 * rng.standard_normal((ny, nx))
    uy = 0.04 * rng.standard_normal((ny, nx))
    o = Oracle(OracleParams(nx=nx, ny=ny, tau=1.0), rho=rho, ux=ux, uy=uy)
    f0 = o.populations()  # equilibrium of the fields, a fixed point of the collision
    o.run(1)
    f1 = o.populations()
    for i in range(9):
        np.testing.assert_allclose(f1[i], np.roll(np.roll(f0[i], EY[i], 0), EX[i], 1),
                                   rtol=0, atol=4e-16)
