"""The power-law fluid of Sec. 5 on the 3D lattices (D3Q19, D3Q27) on the
GPU against the oracle: local tau* from the full 3D non-equilibrium stress,
with BGK and with TRT (tau_minus following tau*), for n = 1/2 (closed form
of the tau* equation) and n = 3/2 (Newton solve), in FP64 to accumulated
rounding, FP32 to the 1e-5 target and FP16 deviations with stochastic
rounding to the reduced-storage target; and the steady clamped channel
against its closed form."""
import numpy as np
import pytest

import closed_forms as cf
from oracle.oracle import Oracle3

pytestmark = pytest.mark.gpu


def _fields(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    s = (nz, ny, nx)
    return (1 + 0.005 * rng.standard_normal(s), 0.02 * rng.standard_normal(s),
            0.01 * rng.standard_normal(s), 0.01 * rng.standard_normal(s))


def _spheres(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    m = np.zeros((nz, ny, nx), np.uint8)
    for _ in range(3):
        c = rng.uniform([0, 0, 0], [nx, ny, nz])
        m[(x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < 9.0] = 1
    return m


TOL = {"f64": 1e-11, "f32": 1e-5, "f16": 1e-3}
LAWS = {0.5: dict(n=0.5, K=0.01, tau_min=0.51, tau_max=2.5),
        1.5: dict(n=1.5, K=0.2, tau_min=0.51, tau_max=2.5)}


@pytest.mark.parametrize("lattice", ["d3q19", "d3q27"])
@pytest.mark.parametrize("storage", list(TOL))
@pytest.mark.parametrize("n", list(LAWS))
@pytest.mark.parametrize("collision", [dict(), dict(collision="trt", magic=3.0 / 16.0)])
def test_power_law_3d_against_oracle(lattice, storage, n, collision):
    from paper_2006_12910_amd import lb
    nx, ny, nz = 70, 13, 21
    kw = dict(g=(2e-5, 0.0, 0.0), walls=(False, False, True), obstacles=_spheres(nx, ny, nz, 3),
              init=_fields(nx, ny, nz, 4), lattice=lattice, power_law=LAWS[n], **collision)
    gpu = lb.Domain3(nx, ny, nz, storage=storage, seed=6, **kw)
    ora = Oracle3(nx, ny, nz, **kw)
    for k in (1, 7, 52):
        gpu.step(k)
        ora.run(k)
        rg, *ug = gpu.moments()
        ro, *uo = ora.moments()
        err = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(ug, uo))
                      / sum((b ** 2).sum() for b in uo))
        print(f"power law {lattice} {storage} n {n} {collision} step {gpu.time}: "
              f"drho {np.abs(rg - ro).max():.2e} err {err:.2e}")
        assert err < TOL[storage], (k, err)
    gpu.close()


@pytest.mark.parametrize("lattice", ["d3q19", "d3q27"])
def test_power_law_3d_clamped_channel(lattice):
    """FP64: walls at z = 0 and nz - 1, force along x, n = 1/2, K = 0.01,
    tau* in [0.51, 2.5]: the steady profile against the closed form with the
    clamp, to the oracle's bound."""
    from paper_2006_12910_amd import lb
    nz, g = 66, 1.66e-5
    d = lb.Domain3(3, 3, nz, g=(g, 0.0, 0.0), walls=(False, False, True), storage="f64",
                   lattice=lattice, power_law=LAWS[0.5])
    d.step(80000)
    u = d.moments()[1][1:-1, 0, 0]
    ref = cf.powerlaw_channel(nz, 0.5, 0.01, g, 0.51, 2.5)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    print(f"power-law channel {lattice}: relative L2 against the closed form {err:.3e}")
    assert err < 2e-3
    d.close()
