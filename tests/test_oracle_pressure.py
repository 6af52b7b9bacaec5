"""Pins of the oracle's Zou-He density boundary (used for the pressure-driven
porous-flow workload): prescribed density and zero transverse velocity at the
faces, continuity, and the Poiseuille profile for the imposed gradient."""
import numpy as np

import closed_forms as cf
from oracle import Oracle, OracleParams
from oracle.oracle import PRESSURE, WALL


def test_faces_hold_prescribed_density():
    o = Oracle(OracleParams(nx=20, ny=12, bc_x=PRESSURE, bc_y=WALL, tau=0.7, rho_in=1.002,
                            rho_out=0.998))
    for _ in range(3):
        o.run(7)
        rho, ux, uy = o.moments()
        np.testing.assert_allclose(rho[1:-1, 0], 1.002, rtol=0, atol=1e-15)
        np.testing.assert_allclose(rho[1:-1, -1], 0.998, rtol=0, atol=1e-15)
        assert np.abs(uy[1:-1, [0, -1]]).max() < 1e-16


def test_pressure_channel_continuity_and_profile():
    nx, ny, tau = 96, 34, 0.8
    o = Oracle(OracleParams(nx=nx, ny=ny, bc_x=PRESSURE, bc_y=WALL, tau=tau, rho_in=1.001,
                            rho_out=0.999)).run(30000)
    rho, ux, uy = o.moments()
    flux = (rho * ux)[1:-1, :].sum(0)
    assert flux.std() / flux.mean() < 1e-8
    W = ny - 2
    dpdx = (1.001 - 0.999) / 3 / (nx - 1)
    umax = dpdx * W * W / (8 * cf.nu_of_tau(tau))
    assert abs(ux[1:-1, nx // 2].max() / umax - 1) < 5e-3
