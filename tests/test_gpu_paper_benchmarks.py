"""The paper's three timing benchmarks (Sec. 6) on their full lattices,
GPU against the FP64 oracle: the stand-in geometry and the parameters the
paper states, stepped a short while from rest (the timing runs of the
benchmark use the same set-up)."""
import numpy as np
import pytest

from helpers import make_pair, velocity_error, velocity_max_error
from paper_2006_12910_amd import inputs

pytestmark = pytest.mark.gpu

# Benchmark 1: tau = 0.636, diagonal body force of components 1e-6 and 1e-5
# (its sign is not given; the flow runs towards y = 0), lateral walls, periodic
# along the flow, LJ strength 20 within 2.5 (Eq. MP2), 45 neutral particles.
B1 = dict(tau=0.636, g=(1e-6, -1e-5), lj=(20.0, 2.5, 0.1))
# Benchmark 2: nu = 0.1 (tau = 0.8), kT = 5e-5, no body force.
B2 = dict(tau=0.8, kT=5e-5)
# Benchmark 3: n = 0.5, xi = 1e-3, the paper's viscosity bounds nu* in
# [1e-5, 0.1] (tau in [0.50003, 0.8]); the body force is not given.
B3 = dict(g=(1e-6, 0.0), power_law=dict(n=0.5, K=1e-3, tau_min=0.50003, tau_max=0.8))


def b1_pair(storage, rounding="nearest"):
    mask, centres = inputs.replica_b1()
    parts = [dict(x=x, y=y, radius=6.5) for x, y in centres]
    return make_pair(1020, 1620, storage=storage, rounding=rounding, bc_x="wall", obstacles=mask,
                     particles=parts, force_average=True, **B1)


def b2_pair(storage):
    ((x, y),) = inputs.replica_b2()
    return make_pair(3000, 41, storage=storage, bc_y="wall", seed=2020, domain_id=2,
                     particles=[dict(x=x, y=y, radius=7.5)], **B2)


def b3_pair(storage, rounding="nearest"):
    return make_pair(101, 51, storage=storage, rounding=rounding, bc_y="wall", tau=0.8, **B3)


def _particles_diff(gpu, ora):
    cols = [0, 1, 4, 5, 6]  # x, y, ux, uy, omega
    return float(np.abs(gpu.particles()[:, cols] - ora.particles()[:, cols]).max())


@pytest.mark.parametrize("storage,rounding,tol,ptol", [("f64", "nearest", 1e-10, 1e-11),
                                                       ("f32", "nearest", 1e-5, 1e-7),
                                                       ("f32", "stochastic", 1e-5, 1e-7)])
def test_b1_porous_particles_against_oracle(storage, rounding, tol, ptol):
    gpu, ora = b1_pair(storage, rounding)
    gpu.step(20)
    ora.run(20)
    drho, err = velocity_error(gpu, ora)
    emax = velocity_max_error(gpu, ora)
    pd = _particles_diff(gpu, ora)
    print(f"B1 {storage}/{rounding}: drho {drho:.2e} err {err:.2e} max {emax:.2e} particles {pd:.2e}",
          flush=True)
    assert err < tol and emax < tol and pd < ptol, (err, emax, pd)


@pytest.mark.parametrize("storage,tol,ptol", [("f64", 1e-10, 1e-11), ("f32", 1e-5, 1e-7)])
def test_b2_brownian_channel_against_oracle(storage, tol, ptol):
    gpu, ora = b2_pair(storage)
    gpu.step(200)
    ora.run(200)
    drho, err = velocity_error(gpu, ora)
    pd = _particles_diff(gpu, ora)
    print(f"B2 {storage}: drho {drho:.2e} err {err:.2e} particles {pd:.2e}", flush=True)
    assert err < tol and pd < ptol, (err, pd)


@pytest.mark.parametrize("storage,rounding,tol", [("f64", "nearest", 1e-10), ("f32", "nearest", 1e-5),
                                                  ("f32", "stochastic", 1e-5)])
def test_b3_powerlaw_channel_against_oracle(storage, rounding, tol):
    gpu, ora = b3_pair(storage, rounding)
    gpu.step(3000)
    ora.run(3000)
    drho, err = velocity_error(gpu, ora)
    print(f"B3 {storage}/{rounding}: drho {drho:.2e} err {err:.2e}", flush=True)
    assert err < tol, err
