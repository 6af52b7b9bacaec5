"""Pins of the oracle's lattice, equilibrium and noise projection.

The equilibrium (Sec. 2, Eq. LB2) is pinned by its exact moments; the noise
projection (Sec. 4, Eq. NP2) by Table t1 as printed in the paper.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import Oracle, OracleParams, normals

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OMEGA = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def load_table_t1():
    rows, wk = [], []
    for line in open(os.path.join(GOLD, "d2q9_table_t1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, vals, w = line.split(":")
        rows.append([int(v) for v in vals.split()])
        wk.append(float(Fraction(w.strip())))
    return np.array(rows, dtype=np.float64), np.array(wk)


def test_table_t1_fixture_consistent_with_weights():
    e, wk = load_table_t1()
    # w_k = sum_i omega_i e_ki^2 (caption of Table t1)
    np.testing.assert_allclose((OMEGA * e * e).sum(1), wk, rtol=0, atol=1e-15)
    chi = e / np.sqrt(wk)[:, None]
    # orthonormality sum_i omega_i chi_ki chi_li = delta_kl
    np.testing.assert_allclose((chi * OMEGA) @ chi.T, np.eye(9), atol=1e-14)
    # completeness omega_i sum_k chi_ki chi_ki' = delta_ii'
    np.testing.assert_allclose(OMEGA[:, None] * (chi.T @ chi), np.eye(9), atol=1e-14)


def test_equilibrium_moments():
    rng = np.random.default_rng(5)
    ny, nx = 6, 7
    rho = 1 + 0.05 * rng.standard_normal((ny, nx))
    ux = 0.05 * rng.standard_normal((ny, nx))
    uy = 0.05 * rng.standard_normal((ny, nx))
    o = Oracle(OracleParams(nx=nx, ny=ny), rho=rho, ux=ux, uy=uy)
    f = o.populations()
    ex, ey = EX[:, None, None], EY[:, None, None]
    np.testing.assert_allclose(f.sum(0), rho, rtol=1e-15)
    np.testing.assert_allclose((f * ex).sum(0), rho * ux, atol=1e-16)
    np.testing.assert_allclose((f * ey).sum(0), rho * uy, atol=1e-16)
    np.testing.assert_allclose((f * ex * ex).sum(0), rho * (ux * ux + 1 / 3), rtol=1e-14)
    np.testing.assert_allclose((f * ey * ey).sum(0), rho * (uy * uy + 1 / 3), rtol=1e-14)
    np.testing.assert_allclose((f * ex * ey).sum(0), rho * ux * uy, atol=1e-16)
    # third-order moment of the D2Q9 equilibrium: sum f ex^2 ey = rho uy / 3
    np.testing.assert_allclose((f * ex * ex * ey).sum(0), rho * uy / 3, atol=1e-16)


@pytest.mark.parametrize("kT", [1e-4, 3e-3])
def test_noise_projection_matches_table_t1(kT):
    """One step from uniform rest at tau = 1 (varpi = 1): f_i(x) at t = 1 is
    omega_i rho0 + zeta_i(x - e_i) with zeta from Eq. NP2 and Table t1."""
    nx, ny, seed = 9, 7, 0xC0FFEE1234
    o = Oracle(OracleParams(nx=nx, ny=ny, tau=1.0, kT=kT, seed=seed, domain_id=3))
    o.run(1)
    f = o.populations()
    e, wk = load_table_t1()
    chi = e / np.sqrt(wk)[:, None]
    amp = np.sqrt(1.0 * kT * 1.0 * (2 - 1.0) / (1 / 3))
    for y in range(ny):
        for x in range(nx):
            th = normals(seed, 3, y * nx + x, 0).astype(np.float64)
            zeta = amp * OMEGA * (chi[3:9].T @ th)
            for i in range(9):
                xd, yd = (x + EX[i]) % nx, (y + EY[i]) % ny
                assert abs(f[i, yd, xd] - (OMEGA[i] + zeta[i])) < 4e-16


def test_noise_conserves_mass_and_momentum():
    o = Oracle(OracleParams(nx=16, ny=12, tau=0.9, kT=1e-3, seed=11))
    m0, j0 = o.mass(), o.momentum()
    o.run(3)
    assert abs(o.mass() / m0 - 1) < 1e-14
    assert max(abs(a - b) for a, b in zip(o.momentum(), j0)) < 1e-14
