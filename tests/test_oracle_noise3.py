"""Pins of the oracle's thermal noise on the 3D lattices (the fluctuating
method of Sec. 4 carried to D3Q19 and D3Q27).  The D2Q9 method draws one
independent unit normal per non-conserved mode of a basis orthonormal in the
weights and scales it by sqrt(rho kT omega (2 - omega) / c_s^2); the oracle
draws the same Gaussian as q weighted normals less their mass and momentum
parts.  Pinned against what that fixes, independently of the oracle's
formula: the noise carries no mass or momentum; on an orthonormal basis of
the non-conserved modes built here (numpy SVD) its coordinates are
uncorrelated with variance 3 kT omega (2 - omega) at rho = 1; and a periodic
box relaxes to equipartition, <rho u_a^2> = kT and <drho^2> = rho kT / c_s^2
= 3 kT; with the two-relaxation-time collision, the even and odd
non-conserved modes each at their own rate's amplitude, uncorrelated, and
the same equipartition.  The normals are the D2Q9 generator's with the Philox counter's third
word as a block index; block 0 is the D2Q9 draw itself."""
import numpy as np
import pytest

from oracle.oracle import Oracle3, lattice3, normals, normals_block

LATTICES = ["d3q19", "d3q27"]
Q = {"d3q19": 19, "d3q27": 27}


def test_block_zero_is_the_d2q9_draw():
    for node, step in [(0, 0), (12345, 7), (2**32 - 1, 2**31)]:
        a = normals(0xDEADBEEF12345678, 0, node, step)
        b = normals_block(0xDEADBEEF12345678, 0, node, step, 0)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        c = normals_block(0xDEADBEEF12345678, 0, node, step, 1)
        assert not np.any(c == b)


def _post_collision(o, q):
    """f* of the last step from f(t+1): f*_i(x) = f_i(x + e_i) (periodic)."""
    ex, ey, ez, _ = lattice3(q)
    f = o.populations()
    return np.stack([np.roll(f[i], (-ez[i], -ey[i], -ex[i]), axis=(0, 1, 2)) for i in range(q)])


@pytest.mark.parametrize("lattice", LATTICES)
def test_noise_conserves_mass_and_momentum(lattice):
    q = Q[lattice]
    n = (10, 9, 8)
    rng = np.random.default_rng(3)
    shape = (n[2], n[1], n[0])
    init = (1 + 0.01 * rng.standard_normal(shape),) + tuple(0.02 * rng.standard_normal(shape) for _ in range(3))
    o = Oracle3(*n, tau=0.8, lattice=lattice, init=init, kT=1e-3, seed=99)
    quiet = Oracle3(*n, tau=0.8, lattice=lattice, init=init)
    m0, j0 = o.mass(), o.momentum()
    o.run(5)
    quiet.run(5)
    assert abs(o.mass() - m0) < 1e-12 * m0
    np.testing.assert_allclose(o.momentum(), j0, rtol=0, atol=1e-12)
    # and the noise is really there: far above round-off against the quiet run
    assert np.abs(o.populations() - quiet.populations()).max() > 1e-4


@pytest.mark.parametrize("lattice", LATTICES)
def test_mode_covariance(lattice):
    """One step from rest at rho = 1, tau = 1: f* = w + zeta at every node."""
    q = Q[lattice]
    ex, ey, ez, w = lattice3(q)
    kT = 1e-4
    n = 32
    o = Oracle3(n, n, n, tau=1.0, lattice=lattice, kT=kT, seed=2024)
    o.run(1)
    zeta = _post_collision(o, q).reshape(q, -1) - w[:, None]
    y = zeta / np.sqrt(w)[:, None]
    cons = np.stack([np.sqrt(w), np.sqrt(w) * ex, np.sqrt(w) * ey, np.sqrt(w) * ez], 1)
    # the conserved coordinates vanish to round-off
    assert np.abs(cons.T @ y).max() < 1e-15
    # an orthonormal basis of the complement: the right singular vectors of
    # the conserved block beyond its rank
    _, _, vt = np.linalg.svd(cons.T)
    basis = vt[4:].T
    assert basis.shape == (q, q - 4)
    c = basis.T @ y
    amp2 = 3 * kT * 1.0 * (2 - 1.0)
    cov = (c @ c.T) / c.shape[1] / amp2
    nsamp = c.shape[1]
    assert np.abs(c.mean(1)).max() < 6 * np.sqrt(amp2 / nsamp)
    assert np.abs(np.diag(cov) - 1).max() < 6 * np.sqrt(2 / nsamp)
    off = cov - np.diag(np.diag(cov))
    assert np.abs(off).max() < 6 * np.sqrt(1 / nsamp)


@pytest.mark.parametrize("lattice", LATTICES)
def test_amplitude_follows_omega(lattice):
    """At tau = 2 the variance is omega (2 - omega) = 3/4 of that at tau = 1."""
    q = Q[lattice]
    _, _, _, w = lattice3(q)
    n = 24
    var = []
    for tau in (1.0, 2.0):
        o = Oracle3(n, n, n, tau=tau, lattice=lattice, kT=1e-4, seed=5)
        o.run(1)
        z = _post_collision(o, q).reshape(q, -1) - w[:, None]
        var.append(float(np.mean(z * z / w[:, None])))
    # identical draws (same seed, node, step): the ratio is exact up to round-off
    assert abs(var[1] / var[0] - 0.75) < 1e-10


@pytest.mark.parametrize("lattice", LATTICES)
def test_equipartition(lattice):
    n, kT = 12, 1e-4
    o = Oracle3(n, n, n, tau=1.0, lattice=lattice, kT=kT, seed=7)
    o.run(300)
    ju, dr = [], []
    for _ in range(100):
        o.run(4)
        rho, ux, uy, uz = o.moments()
        ju.append([np.mean(rho * u * u) for u in (ux, uy, uz)])
        dr.append(np.mean((rho - 1.0) ** 2))
    t = np.mean(ju, 0) / kT
    assert np.abs(t - 1).max() < 0.03, t
    assert abs(np.mean(dr) / (3 * kT) - 1) < 0.03, np.mean(dr) / (3 * kT)


def _parity_bases(q, ex, ey, ez, w):
    """Orthonormal bases (in zeta / sqrt(w) coordinates) of the non-conserved
    modes even and odd under e -> -e: the even ones orthogonal to sqrt(w),
    the odd ones to sqrt(w) e."""
    pairs = [(i, i + 1) for i in range(1, q, 2)]
    bs = np.zeros((q, len(pairs) + 1))
    bs[0, 0] = 1.0
    ba = np.zeros((q, len(pairs)))
    for k, (i, j) in enumerate(pairs):
        bs[i, k + 1] = bs[j, k + 1] = np.sqrt(0.5)
        ba[i, k], ba[j, k] = np.sqrt(0.5), -np.sqrt(0.5)
    sw = np.sqrt(w)
    _, _, v = np.linalg.svd((bs.T @ sw)[None, :])
    even = bs @ v[1:].T
    _, _, v = np.linalg.svd((ba.T @ np.stack([sw * ex, sw * ey, sw * ez], 1)).T)
    odd = ba @ v[3:].T
    return even, odd


@pytest.mark.parametrize("lattice", LATTICES)
def test_trt_mode_covariance_per_parity(lattice):
    """With TRT the even non-conserved modes carry omega (2 - omega) at
    omega = 1/tau and the odd ones at 1/tau_minus: tau = 1.5, magic 0.05
    (tau_minus = 0.55) makes them 0.889 and 0.331.  One step from rest:
    f* = w + zeta."""
    q = Q[lattice]
    ex, ey, ez, w = lattice3(q)
    kT, tau, magic = 1e-4, 1.5, 0.05
    n = 32
    o = Oracle3(n, n, n, tau=tau, lattice=lattice, kT=kT, seed=77, collision="trt", magic=magic)
    o.run(1)
    y = (_post_collision(o, q).reshape(q, -1) - w[:, None]) / np.sqrt(w)[:, None]
    even, odd = _parity_bases(q, ex, ey, ez, w)
    assert even.shape[1] + odd.shape[1] == q - 4
    tm = 0.5 + magic / (tau - 0.5)
    nsamp = y.shape[1]
    for basis, om in ((even, 1 / tau), (odd, 1 / tm)):
        c = basis.T @ y
        cov = (c @ c.T) / nsamp / (3 * kT * om * (2 - om))
        assert np.abs(np.diag(cov) - 1).max() < 6 * np.sqrt(2 / nsamp)
        assert np.abs(cov - np.diag(np.diag(cov))).max() < 6 * np.sqrt(1 / nsamp)
    cross = (even.T @ y) @ (odd.T @ y).T / nsamp / (3 * kT)
    assert np.abs(cross).max() < 6 * np.sqrt(1 / nsamp)


@pytest.mark.parametrize("lattice", LATTICES)
def test_trt_equipartition(lattice):
    n, kT = 12, 1e-4
    o = Oracle3(n, n, n, tau=1.0, lattice=lattice, kT=kT, seed=11, collision="trt", magic=0.05)
    o.run(300)
    ju, dr = [], []
    for _ in range(100):
        o.run(4)
        rho, ux, uy, uz = o.moments()
        ju.append([np.mean(rho * u * u) for u in (ux, uy, uz)])
        dr.append(np.mean((rho - 1.0) ** 2))
    t = np.mean(ju, 0) / kT
    assert np.abs(t - 1).max() < 0.03, t
    assert abs(np.mean(dr) / (3 * kT) - 1) < 0.03, np.mean(dr) / (3 * kT)


def test_rejects_negative_kT():
    with pytest.raises(ValueError):
        Oracle3(8, 8, 8, kT=-1e-4)
    with pytest.raises(ValueError):
        Oracle3(8, 8, 8, collision="trt", kT=-1e-4)
