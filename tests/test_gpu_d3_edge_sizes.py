"""The 3D sweeps at degenerate sizes against the oracle: the smallest lattice
(3 x 3 x 3, where x - 1 and x + 1 both wrap and most lanes of the 64 x 4
tile are idle), one node past a full tile in x, and a thin z extent; every
feature (BGK, TRT, thermal noise with either, power law) on both lattices, FP64 to
accumulated rounding, FP32 to the 1e-5 target, FP16 deviations with
stochastic rounding to the 1e-3 target."""
import numpy as np
import pytest

from oracle.oracle import Oracle3

pytestmark = pytest.mark.gpu

SHAPES = [(3, 3, 3), (65, 3, 4), (5, 6, 3)]
FEATURES = {
    "bgk": dict(),
    "trt": dict(collision="trt", magic=3.0 / 16.0),
    "noise": dict(kT=1e-4, seed=8),
    "trt_noise": dict(collision="trt", magic=0.05, kT=1e-4, seed=9),
    "power": dict(power_law=dict(n=0.75, K=0.01)),
}
TOL = {"f64": 1e-11, "f32": 1e-5, "f16": 1e-3}


@pytest.mark.parametrize("storage", list(TOL))
@pytest.mark.parametrize("feature", list(FEATURES))
@pytest.mark.parametrize("lattice", ["d3q19", "d3q27"])
@pytest.mark.parametrize("shape", SHAPES)
def test_d3_edge_sizes_against_oracle(shape, lattice, feature, storage):
    from paper_2006_12910_amd import lb
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    s = (nz, ny, nx)
    init = (1 + 0.003 * rng.standard_normal(s),) + tuple(0.01 * rng.standard_normal(s) for _ in range(3))
    kw = dict(tau=0.8, g=(1e-5, 2e-6, -3e-6), lattice=lattice, init=init, **FEATURES[feature])
    if nx > 3:  # one solid node away from the edges of the smallest lattices
        mask = np.zeros(s, np.uint8)
        mask[1, 1, 1] = 1
        kw["obstacles"] = mask
    gpu = lb.Domain3(nx, ny, nz, storage=storage, **kw)
    ora = Oracle3(nx, ny, nz, **kw)
    gpu.step(12)
    ora.run(12)
    rg, *ug = gpu.moments()
    ro, *uo = ora.moments()
    err = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(ug, uo))) / np.sqrt(sum((b ** 2).sum() for b in uo))
    drho = np.abs(rg - ro).max()
    print(f"{shape} {lattice} {feature} {storage}: drho {drho:.2e} err {err:.2e}")
    assert err < TOL[storage]
    assert drho < {"f64": 1e-13, "f32": 1e-6, "f16": 1e-4}[storage]
    gpu.close()
