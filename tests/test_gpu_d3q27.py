"""GPU vs oracle parity of the D3Q27 sweep (the second 3D lattice the
paper's outlook points to, Sec. 8; BGK with the velocity-shift forcing of
Sec. 2, and the two-relaxation-time variant): FP64 storage to accumulated
rounding and FP32 to the 1e-5 target on ragged
lattices with walls and spherical obstacles; FP16 / BF16 deviation storage
to the reduced-storage targets; the exact discrete plane Poiseuille state
(BGK) and the walls exactly halfway (TRT, magic 3/16); the 64-bit-offset
sweep bit-identical to the 32-bit one; the closed-form shear-wave decay and
the mass at the benchmark size (256^3)."""
import numpy as np
import pytest

from oracle.oracle import Oracle3

pytestmark = pytest.mark.gpu


def _spheres(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    m = np.zeros((nz, ny, nx), np.uint8)
    for _ in range(4):
        c = rng.uniform([0, 0, 0], [nx, ny, nz])
        r = rng.uniform(2.0, 4.5)
        m[(x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < r * r] = 1
    return m


def _fields(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    s = (nz, ny, nx)
    return (1 + 0.005 * rng.standard_normal(s), 0.02 * rng.standard_normal(s),
            0.02 * rng.standard_normal(s), 0.02 * rng.standard_normal(s))


def _velocity_error(gpu, ora):
    rg, *ug = gpu.moments()
    ro, *uo = ora.moments()
    num = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(ug, uo)))
    den = np.sqrt(sum((b ** 2).sum() for b in uo))
    return np.abs(rg - ro).max(), num / den


TOL = {("f64", None): 1e-11, ("f32", None): 1e-5, ("f16", "stochastic"): 1e-3,
       ("bf16", "stochastic"): 1e-2}


@pytest.mark.parametrize("storage,rounding", list(TOL))
@pytest.mark.parametrize("shape", [(70, 33, 21), (130, 7, 5)])
@pytest.mark.parametrize("collision", [dict(), dict(collision="trt", magic=3.0 / 16.0)])
def test_d3q27_against_oracle(storage, rounding, shape, collision):
    from paper_2006_12910_amd import lb
    nx, ny, nz = shape
    mask = _spheres(nx, ny, nz, nx + ny)
    init = _fields(nx, ny, nz, nz)
    kw = dict(tau=0.7, g=(2e-5, -1e-5, 5e-6), walls=(False, False, True), **collision)
    gpu = lb.Domain3(nx, ny, nz, storage=storage, rounding=rounding, seed=13, obstacles=mask,
                     init=init, lattice="d3q27", **kw)
    ora = Oracle3(nx, ny, nz, obstacles=mask, init=init, lattice="d3q27", **kw)
    tol = TOL[(storage, rounding)]
    for n in (1, 7, 52):
        gpu.step(n)
        ora.run(n)
        drho, err = _velocity_error(gpu, ora)
        print(f"D3Q27 {storage} {shape} {collision} step {gpu.time}: drho {drho:.2e} err {err:.2e}")
        assert err < tol, (n, drho, err)
        assert drho < {"f64": 1e-13, "f32": 1e-6, "f16": 2e-4, "bf16": 2e-3}[storage]
    m_gpu, m_ora = gpu.mass(), ora.mass()
    # FP64 mass: 16-bit stochastic rounding walks it randomly (BF16 spacing
    # is 8 x FP16's), FP32 holds it to its summation rounding
    assert abs(m_gpu - m_ora) / m_ora < {"f64": 1e-13, "f32": 1e-7, "f16": 1e-6, "bf16": 1e-5}[storage]
    gpu.close()


def test_d3q27_plane_poiseuille_exact_steady_state_and_trt_walls():
    """FP64: BGK reaches the exact discrete steady profile (the D2Q9 one:
    D3Q27 sums over e_y to D2Q9), TRT with magic 3/16 the parabola with the
    walls exactly halfway."""
    from paper_2006_12910_amd import lb
    nz, g = 34, 1e-6
    z = np.arange(1, nz - 1)
    for tau, coll in ((0.8, dict()), (1.8, dict(collision="trt", magic=3.0 / 16.0))):
        gpu = lb.Domain3(64, 4, nz, tau=tau, g=(g, 0.0, 0.0), walls=(False, False, True),
                         storage="f64", lattice="d3q27", **coll)
        gpu.step(30000)
        _, ux, _, _ = gpu.moments()
        nu = (tau - 0.5) / 3
        ref = g / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
        if not coll:
            ref = ref + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
        dev = np.abs(ux[1:-1] - ref[:, None, None]).max() / ref.max()
        print(f"D3Q27 plane Poiseuille tau {tau} {coll}: max deviation {dev:.2e}")
        assert dev < 1e-10
        gpu.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_d3q27_wide_offsets_give_identical_states(storage):
    from paper_2006_12910_amd import lb
    nx, ny, nz = 70, 33, 21
    kw = dict(tau=0.7, g=(2e-5, -1e-5, 5e-6), storage=storage, seed=4, init=_fields(nx, ny, nz, 8),
              walls=(False, True, False), obstacles=_spheres(nx, ny, nz, 5), lattice="d3q27")
    a = lb.Domain3(nx, ny, nz, **kw)
    b = lb.Domain3(nx, ny, nz, **kw).set_option(lb.LB3_OPT_WIDE_OFFSETS, 1)
    a.step(9)
    b.step(9)
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_d3q27_256_cube_shear_wave_and_mass(storage):
    """The benchmark lattice: a shear wave decays as exp(-nu k^2 t) and the
    FP64 mass sum holds (exactly up to FP32 summation for FP32 storage, the
    random walk of stochastic rounding for FP16)."""
    from paper_2006_12910_amd import lb
    n, u0, tau, steps = 256, 0.01, 0.8, 300
    k = 2 * np.pi / n
    z = np.arange(n)[:, None, None] + np.zeros((1, n, n))
    gpu = lb.Domain3(n, n, n, tau=tau, storage=storage, seed=9, lattice="d3q27",
                     init=(1.0, u0 * np.sin(k * z), 0.0, 0.0))
    m0 = gpu.mass()
    gpu.step(steps)
    _, ux, uy, uz = gpu.moments()
    prof = ux.mean(axis=(1, 2))
    amp = 2 * (prof * np.sin(k * np.arange(n))).mean()
    ref = u0 * np.exp(-(tau - 0.5) / 3 * k * k * steps)
    cross = max(np.abs(uy).max(), np.abs(uz).max())
    drift = gpu.mass() / m0 - 1
    print(f"D3Q27 256^3 {storage} shear wave: amplitude / closed form - 1 = {amp / ref - 1:.2e}, "
          f"max cross flow {cross:.2e}, mass drift {drift:.2e}")
    assert abs(amp / ref - 1) < 1e-3
    assert cross < (1e-7 if storage == "f32" else 2e-5)
    assert abs(drift) < (1e-9 if storage == "f32" else 1e-7)
    gpu.close()
