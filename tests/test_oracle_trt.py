"""Pins of the oracle's two-relaxation-time (TRT) collision on D2Q9 (an
addition to the paper's BGK collision of Sec. 2: the parts of each
population pair symmetric and antisymmetric under e -> -e relax with 1/tau
and 1/tau_minus, (tau - 1/2)(tau_minus - 1/2) = magic, and the body force
shifts u_eq by tau_minus g): its reduction to BGK at magic = (tau - 1/2)^2,
exact conservation of mass and of the momentum input g per unit mass, and
the plane Poiseuille profile with the walls exactly halfway at magic = 3/16
for any tau (where BGK keeps a tau-dependent slip)."""
import numpy as np
import pytest

from oracle.oracle import PERIODIC, WALL, Oracle, OracleParams


def _fields(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return (1 + 0.01 * rng.standard_normal((ny, nx)), 0.02 * rng.standard_normal((ny, nx)),
            0.02 * rng.standard_normal((ny, nx)))


def _disc_mask(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx]
    return ((x - nx / 3) ** 2 + (y - ny / 2) ** 2 < 16).astype(np.uint8)


def test_trt_with_the_bgk_magic_number_is_bgk():
    nx, ny, tau = 31, 22, 0.83
    rho, ux, uy = _fields(nx, ny, 1)
    mask = _disc_mask(nx, ny)
    kw = dict(nx=nx, ny=ny, bc_y=WALL, tau=tau, gx=1e-5, gy=-2e-6)
    a = Oracle(OracleParams(**kw), mask, rho, ux, uy)
    b = Oracle(OracleParams(**kw, trt=True, magic=(tau - 0.5) ** 2), mask, rho, ux, uy)
    a.run(60)
    b.run(60)
    assert np.abs(a.populations() - b.populations()).max() < 1e-15


@pytest.mark.parametrize("power_law", [False, True])
def test_trt_conserves_mass_and_adds_the_body_force(power_law):
    nx, ny = 24, 18
    rho, ux, uy = _fields(nx, ny, 2)
    g = np.array([2e-5, -1e-5])
    extra = dict(power_law=True, n_index=0.5, K=0.01) if power_law else dict(tau=0.62)
    o = Oracle(OracleParams(nx=nx, ny=ny, gx=g[0], gy=g[1], trt=True, magic=0.25, **extra),
               None, rho, ux, uy)
    m0 = o.populations().sum()
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    for _ in range(5):
        f0 = o.populations()
        o.run(1)
        f1 = o.populations()
        m = f1.sum()
        dj = np.array([np.einsum("i,i...->...", ex, f1 - f0).sum(), np.einsum("i,i...->...", ey, f1 - f0).sum()])
        np.testing.assert_allclose(dj, g * m, rtol=1e-10, atol=1e-15)
    assert abs(o.populations().sum() - m0) / m0 < 1e-14


def test_trt_magic_3_16_puts_the_poiseuille_walls_exactly_halfway():
    """Walls at y = 0 and ny - 1 (solid rows, halfway bounce-back), force
    along x: with magic 3/16 the steady u = j/rho + g/2 is the parabola
    g/(2 nu) (y - 1/2)(ny - 3/2 - y), nu = (tau - 1/2)/3, to rounding, for
    every tau; BGK at tau = 1.8 is off by its slip term."""
    ny, g = 34, 1e-6
    y = np.arange(1, ny - 1)
    for tau in (0.7, 1.0, 1.8):
        nu = (tau - 0.5) / 3
        parabola = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
        o = Oracle(OracleParams(nx=3, ny=ny, bc_x=PERIODIC, bc_y=WALL, tau=tau, gx=g, trt=True,
                                magic=3.0 / 16.0))
        o.run(50000 if tau < 0.8 else 30000)
        _, u, _ = o.moments()
        dev = np.abs(u[1:-1, :] - parabola[:, None]).max() / parabola.max()
        assert dev < 1e-10, (tau, dev)
    o = Oracle(OracleParams(nx=3, ny=ny, bc_x=PERIODIC, bc_y=WALL, tau=1.8, gx=g))
    o.run(30000)
    _, u, _ = o.moments()
    nu = 1.3 / 3
    parabola = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    assert np.abs(u[1:-1, :] - parabola[:, None]).max() / parabola.max() > 1e-3


def test_trt_with_noise_is_rejected():
    with pytest.raises(ValueError):
        Oracle(OracleParams(nx=8, ny=8, kT=1e-5, trt=True))
