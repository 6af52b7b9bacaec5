"""Pins of the oracle's three-dimensional variants, D3Q19 and D3Q27 (the 3D
lattices the paper names as its next step, Sec. 8, with the BGK collision
and the velocity-shift forcing of Sec. 2): lattice isotropy, equilibrium
moments, exact conservation, the exact discrete steady solution of plane
Poiseuille flow, shear-wave decay at the BGK viscosity, the series solution
of square-duct flow with second-order convergence, and flows uniform along
y that equal the independent D2Q9 oracle's step for step (both lattices
project onto D2Q9); for the two-relaxation-time variant, its reduction to
BGK, its conservation and the walls exactly halfway at the magic number
3/16; for the power law of Sec. 5 on the 3D lattices, n = 1 equal to the
Newtonian run, a flow uniform along y on D3Q27 equal to the D2Q9 oracle's
power-law step (the tensor-product lattice leaves the y rows of the stress
at equilibrium), and the clamped channel against its closed form."""
import numpy as np
import pytest

import closed_forms as cf

from oracle.oracle import PERIODIC, WALL, Oracle, Oracle3, OracleParams, lattice3

LATTICES = ["d3q19", "d3q27"]
Q = {"d3q19": 19, "d3q27": 27}


@pytest.mark.parametrize("lattice", LATTICES)
def test_lattice_isotropy(lattice):
    q = Q[lattice]
    ex, ey, ez, w = lattice3(q)
    e = np.stack([ex, ey, ez], 1)
    assert len({tuple(v) for v in e}) == q
    assert sorted((e ** 2).sum(1).tolist()) == [0] + [1] * 6 + [2] * 12 + ([3] * 8 if q == 27 else [])
    if q == 27:  # weights of the tensor-product lattice
        np.testing.assert_allclose(sorted(set(np.round(w, 15))), [1 / 216, 1 / 54, 2 / 27, 8 / 27])
    for i in range(1, q):  # opposites pair as (i, i + 1), i odd
        j = i + 1 if i % 2 else i - 1
        assert np.array_equal(e[j], -e[i])
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", w, e, e)
    np.testing.assert_allclose(m2, d / 3, atol=1e-15)
    assert np.abs(np.einsum("i,ia->a", w, e)).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, e, e, e)).max() < 1e-15
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(m4, iso, atol=1e-15)


@pytest.mark.parametrize("lattice", LATTICES)
def test_equilibrium_moments(lattice):
    """Populations of the initial state (equilibria) have density rho,
    momentum rho u and momentum flux rho/3 I + rho u u."""
    rng = np.random.default_rng(3)
    shape = (5, 4, 6)
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = 0.05 * rng.standard_normal((3,) + shape)
    o = Oracle3(6, 4, 5, init=(rho, u[0], u[1], u[2]), lattice=lattice)
    f = o.populations()
    ex, ey, ez, _ = lattice3(Q[lattice])
    e = np.stack([ex, ey, ez], 1).astype(float)
    np.testing.assert_allclose(f.sum(0), rho, rtol=1e-14)
    j = np.einsum("ia,i...->a...", e, f)
    np.testing.assert_allclose(j, rho * u, atol=1e-15)
    pi = np.einsum("ia,ib,i...->ab...", e, e, f)
    ref = np.einsum("ab,...->ab...", np.eye(3), rho / 3) + rho * np.einsum("a...,b...->ab...", u, u)
    np.testing.assert_allclose(pi, ref, atol=1e-14)


@pytest.mark.parametrize("lattice", LATTICES)
def test_mass_and_momentum_balance(lattice):
    """Periodic box with an obstacle: mass is conserved and the momentum
    grows by g times the fluid mass each step, less what the solid takes."""
    rng = np.random.default_rng(4)
    n = (10, 9, 8)
    o = Oracle3(*n, tau=0.7, g=(2e-5, -1e-5, 3e-6), lattice=lattice,
                init=(1 + 0.01 * rng.standard_normal(n[::-1]), 0.01 * rng.standard_normal(n[::-1]),
                      0.0, 0.0))
    m0 = o.mass()
    o.run(40)
    assert abs(o.mass() - m0) / m0 < 1e-13
    free = Oracle3(*n, tau=0.7, g=(2e-5, -1e-5, 3e-6), lattice=lattice)
    for _ in range(5):
        j0 = free.momentum()
        free.run(1)
        np.testing.assert_allclose(free.momentum() - j0, np.array([2e-5, -1e-5, 3e-6]) * free.mass(),
                                   rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("lattice", LATTICES)
def test_plane_poiseuille_exact_discrete_steady_state(lattice):
    """Walls at z = 0 and nz - 1 (halfway bounce-back), body force along x:
    the steady u = j/rho + g/2 is the exact discrete solution
    g/(2 nu) (z - 1/2)(nz - 3/2 - z) + g (16 (tau - 1/2)^2 - 3) / (24 nu),
    the same as on D2Q9 (the flow involves only the populations with
    e_z != 0, which bounce back alike)."""
    nz, g, tau = 34, 1e-6, 0.8
    o = Oracle3(4, 4, nz, tau=tau, g=(g, 0.0, 0.0), walls=(False, False, True), lattice=lattice)
    o.run(30000)
    _, ux, uy, uz = o.moments()
    nu = (tau - 0.5) / 3
    z = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (z - 0.5) * (nz - 1.5 - z) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    u = ux[1:-1, :, :]
    assert np.abs(u - exact[:, None, None]).max() / exact.max() < 1e-10
    assert max(np.abs(uy).max(), np.abs(uz).max()) < 1e-10 * exact.max()


@pytest.mark.parametrize("lattice", LATTICES)
def test_shear_wave_decays_at_the_bgk_viscosity(lattice):
    """u_x = u0 sin(k z) in a periodic box decays as exp(-nu k^2 t) with
    nu = (tau - 1/2)/3, up to O(k^2) lattice corrections."""
    nz, u0, t = 64, 1e-3, 600
    k = 2 * np.pi / nz
    for tau in (0.6, 1.1):
        z = np.arange(nz)[:, None, None] + np.zeros((nz, 3, 4))
        o = Oracle3(4, 3, nz, tau=tau, init=(1.0, u0 * np.sin(k * z), 0.0, 0.0), lattice=lattice)
        o.run(t)
        _, ux, _, _ = o.moments()
        amp = 2 * (ux[:, 0, 0] * np.sin(k * np.arange(nz))).mean()
        ref = u0 * np.exp(-(tau - 0.5) / 3 * k * k * t)
        assert abs(amp / ref - 1) < 2e-3, (tau, amp, ref)


def _duct_series(n, g, nu, terms=200):
    """Square duct, walls halfway between the solid planes: half width
    a = (n - 2)/2; u = 16 a^2 g/(nu pi^3) sum_(m odd) (-1)^((m-1)/2) m^-3
    [1 - cosh(m pi z/(2a)) / cosh(m pi/2)] cos(m pi y/(2a))."""
    a = (n - 2) / 2.0
    c = np.arange(n) - (n - 1) / 2.0
    Z, Y = np.meshgrid(c, c, indexing="ij")
    u = np.zeros_like(Y)
    for q in range(terms):
        m = 2 * q + 1
        u += (-1) ** q / m ** 3 * (1 - np.cosh(m * np.pi * Z / (2 * a)) / np.cosh(m * np.pi / 2)) \
            * np.cos(m * np.pi * Y / (2 * a))
    return 16 * a * a * g / (nu * np.pi ** 3) * u


def test_square_duct_flow_converges_to_the_series_solution():
    g, tau = 1e-6, 0.8
    nu = (tau - 0.5) / 3
    errs = []
    for n in (18, 34):
        o = Oracle3(4, n, n, tau=tau, g=(g, 0.0, 0.0), walls=(False, True, True))
        o.run(int(4 * n * n / nu))
        _, ux, _, _ = o.moments()
        u = ux[1:-1, 1:-1, 0]
        ref = _duct_series(n, g, nu)[1:-1, 1:-1]
        errs.append(np.sqrt(((u - ref) ** 2).sum() / (ref ** 2).sum()))
    assert errs[1] < 1.5e-3
    assert errs[0] / errs[1] > 3.0  # second order in the lattice spacing


@pytest.mark.parametrize("lattice", LATTICES)
def test_y_uniform_flow_equals_the_d2q9_oracle(lattice):
    """A flow uniform along y: summing D3Q19 or D3Q27 over e_y gives the
    D2Q9 velocity set with its weights (4/9, 1/9, 1/36), and the summed
    equilibrium is the D2Q9 one when u_y = 0, so the 3D step reduces to the
    D2Q9 step in the (x, z) plane.  Checked against the D2Q9 oracle (its
    own code, pinned on its own): an obstacle extruded along y, walls at
    z = 0 and nz - 1, a body force in x and z, random initial fields."""
    rng = np.random.default_rng(21)
    nx, ny, nz = 23, 3, 17
    X, Z = np.meshgrid(np.arange(nx), np.arange(nz))
    mask2 = ((X - 9.3) ** 2 + (Z - 8.1) ** 2 < 9.0).astype(np.uint8)
    rho2 = 1 + 0.01 * rng.standard_normal((nz, nx))
    ux2, uz2 = 0.02 * rng.standard_normal((2, nz, nx))
    g = (3e-5, 0.0, -2e-5)
    ext = lambda a: np.repeat(a[:, None, :], ny, axis=1)  # [nz][nx] -> [nz][ny][nx]
    o3 = Oracle3(nx, ny, nz, tau=0.73, g=g, walls=(False, False, True), obstacles=ext(mask2),
                 init=(ext(rho2), ext(ux2), 0.0, ext(uz2)), lattice=lattice)
    o2 = Oracle(OracleParams(nx=nx, ny=nz, bc_x=PERIODIC, bc_y=WALL, tau=0.73, gx=g[0], gy=g[2]),
                obstacles=mask2, rho=rho2, ux=ux2, uy=uz2)
    for n in (1, 9, 90):
        o3.run(n)
        o2.run(n)
        r3, u3, v3, w3 = o3.moments()
        r2, u2, w2 = o2.moments()
        for a, b in ((r3, r2), (u3, u2), (w3, w2)):
            for y in range(ny):
                assert np.abs(a[:, y, :] - b).max() < 1e-13, (lattice, n)
        assert np.abs(v3).max() < 1e-16


# --- two-relaxation-time (TRT) collision ----------------------------------

def test_trt_with_the_bgk_magic_number_is_bgk():
    """With magic = (tau - 1/2)^2 the antisymmetric parts relax at 1/tau too:
    the TRT collision is the BGK one (only the rounding order differs)."""
    rng = np.random.default_rng(11)
    n = (9, 7, 6)
    init = (1 + 0.01 * rng.standard_normal(n[::-1]), 0.02 * rng.standard_normal(n[::-1]),
            0.01 * rng.standard_normal(n[::-1]), 0.0)
    tau = 0.83
    a = Oracle3(*n, tau=tau, g=(1e-5, 0.0, -2e-6), walls=(False, True, False), init=init)
    b = Oracle3(*n, tau=tau, g=(1e-5, 0.0, -2e-6), walls=(False, True, False), init=init,
                collision="trt", magic=(tau - 0.5) ** 2)
    a.run(50)
    b.run(50)
    assert np.abs(a.populations() - b.populations()).max() < 1e-15


def test_trt_conserves_mass_and_adds_the_body_force():
    """The TRT step conserves mass and adds g times the fluid mass to the
    momentum each step (the force shifts u_eq by tau_minus g, and only the
    antisymmetric parts carry momentum)."""
    rng = np.random.default_rng(12)
    n = (10, 9, 8)
    g = np.array([2e-5, -1e-5, 3e-6])
    o = Oracle3(*n, tau=0.62, g=tuple(g), collision="trt", magic=0.25,
                init=(1 + 0.01 * rng.standard_normal(n[::-1]), 0.01 * rng.standard_normal(n[::-1]),
                      0.005 * rng.standard_normal(n[::-1]), 0.0))
    m0 = o.mass()
    for _ in range(5):
        j0 = o.momentum()
        o.run(1)
        np.testing.assert_allclose(o.momentum() - j0, g * o.mass(), rtol=1e-11, atol=1e-14)
    assert abs(o.mass() - m0) / m0 < 1e-14


@pytest.mark.parametrize("lattice", LATTICES)
def test_trt_magic_3_16_puts_the_poiseuille_walls_exactly_halfway(lattice):
    """TRT with magic = 3/16 and halfway bounce-back gives plane Poiseuille
    flow with the walls exactly halfway between the solid and the first fluid
    plane, whatever tau (Ginzburg and d'Humieres' result for the TRT
    bounce-back): the steady profile is the parabola
    g/(2 nu) (z - 1/2)(nz - 3/2 - z), nu = (tau - 1/2)/3, with no slip term.
    BGK (magic = (tau - 1/2)^2) keeps a tau-dependent slip, which this
    check also sees."""
    nz, g = 34, 1e-6
    z = np.arange(1, nz - 1)
    for tau in (0.7, 0.9, 1.8):
        nu = (tau - 0.5) / 3
        parabola = g / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
        o = Oracle3(4, 4, nz, tau=tau, g=(g, 0.0, 0.0), walls=(False, False, True),
                    collision="trt", magic=3.0 / 16.0, lattice=lattice)
        o.run(50000 if tau < 0.8 else 30000)  # to steady state: ~ nz^2 / (pi^2 nu) per e-fold
        _, ux, _, _ = o.moments()
        dev = np.abs(ux[1:-1] - parabola[:, None, None]).max() / parabola.max()
        assert dev < 1e-10, (tau, dev)
    # BGK at tau = 1.8: slip g (16 (tau - 1/2)^2 - 3)/(24 nu) ~ 1e-2 of the peak
    o = Oracle3(4, 4, nz, tau=1.8, g=(g, 0.0, 0.0), walls=(False, False, True), lattice=lattice)
    o.run(30000)
    _, ux, _, _ = o.moments()
    nu = 1.3 / 3
    parabola = g / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
    assert np.abs(ux[1:-1] - parabola[:, None, None]).max() / parabola.max() > 1e-3


# --- power law (Sec. 5) on the 3D lattices ---------------------------------

@pytest.mark.parametrize("lattice", LATTICES)
def test_power_law_with_n_1_is_the_newtonian_run(lattice):
    rng = np.random.default_rng(31)
    n = (9, 7, 6)
    init = (1 + 0.01 * rng.standard_normal(n[::-1]), 0.02 * rng.standard_normal(n[::-1]), 0.0,
            0.01 * rng.standard_normal(n[::-1]))
    kw = dict(g=(1e-5, 0.0, -2e-6), walls=(False, True, False), init=init, lattice=lattice)
    a = Oracle3(*n, tau=0.5 + 3 * 0.01, **kw)
    b = Oracle3(*n, power_law=dict(n=1.0, K=0.01), **kw)
    a.run(30)
    b.run(30)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("n", [0.5, 1.5])
def test_d3q27_y_uniform_power_law_flow_equals_the_d2q9_oracle(n):
    """D3Q27 summed over e_y is D2Q9 with its weights, and on a flow uniform
    along y its non-equilibrium stress has no y components, so tau* and the
    whole step equal the D2Q9 power-law step (D3Q19, not a tensor product,
    develops a y y stress and differs at O(1e-4) for n = 1/2)."""
    rng = np.random.default_rng(22)
    nx, ny, nz = 23, 3, 17
    rho2 = 1 + 0.01 * rng.standard_normal((nz, nx))
    ux2, uz2 = 0.02 * rng.standard_normal((2, nz, nx))
    ext = lambda a: np.repeat(a[:, None, :], ny, axis=1)
    pl = dict(n=n, K=0.01, tau_min=0.51, tau_max=2.5)
    o3 = Oracle3(nx, ny, nz, g=(3e-5, 0.0, -2e-5), walls=(False, False, True), lattice="d3q27",
                 init=(ext(rho2), ext(ux2), 0.0, ext(uz2)), power_law=pl)
    o2 = Oracle(OracleParams(nx=nx, ny=nz, bc_y=WALL, gx=3e-5, gy=-2e-5, power_law=True,
                             n_index=n, K=0.01, tau_min=0.51, tau_max=2.5), None, rho2, ux2, uz2)
    for k in (1, 9, 90):
        o3.run(k)
        o2.run(k)
        r3, u3, v3, w3 = o3.moments()
        r2, u2, w2 = o2.moments()
        for a, b in ((r3, r2), (u3, u2), (w3, w2)):
            for y in range(ny):
                assert np.abs(a[:, y, :] - b).max() < 1e-13, (n, k)


@pytest.mark.parametrize("lattice", LATTICES)
def test_clamped_power_law_channel(lattice):
    """Walls at z = 0 and nz - 1, force along x, n = 1/2, K = 0.01, tau* in
    [0.51, 2.5]: the steady profile against the closed form with the clamp,
    to the 2D oracle's bound."""
    nz, g = 66, 1.66e-5
    o = Oracle3(3, 3, nz, g=(g, 0.0, 0.0), walls=(False, False, True), lattice=lattice,
                power_law=dict(n=0.5, K=0.01, tau_min=0.51, tau_max=2.5)).run(80000)
    u = o.moments()[1][1:-1, 0, 0]
    ref = cf.powerlaw_channel(nz, 0.5, 0.01, g, 0.51, 2.5)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err < 2e-3, err
