"""The two-relaxation-time collision of the 2D domains (an addition to the
paper's BGK collision of Sec. 2) on the GPU against the oracle: channels
with walls and obstacles, the power law (tau_minus from the local tau*),
density faces and a moving disc, in FP64 to accumulated rounding and FP32
to the 1e-5 target; two-step launches bit-identical to single steps in
every storage format; the plane Poiseuille parabola with the walls exactly
halfway at magic 3/16."""
import numpy as np
import pytest

from helpers import make_pair, random_fields, velocity_error, velocity_max_error
from paper_2006_12910_amd import inputs, lb

pytestmark = pytest.mark.gpu


def _mask(nx, ny, seed):
    m, _ = inputs.rsa_discs(nx, ny, 3.0, 6.0, 0.15, 1.0, inputs.rng(seed), periodic=True)
    return m


CASES = {
    "channel": dict(bc_y="wall", tau=0.7, g=(3e-6, -1e-6)),
    "obstacles": dict(tau=0.62, g=(2e-6, 1e-6), obstacles=True),
    "power_law": dict(bc_y="wall", g=(4e-6, 0.0),
                      power_law=dict(n=0.5, K=0.01, tau_min=0.51, tau_max=2.5)),
    "pressure": dict(bc_x="pressure", bc_y="wall", tau=0.8, rho_in=1.001, rho_out=0.999),
}


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.4])
def test_trt_against_oracle(storage, tol, case, magic):
    kw = dict(CASES[case])
    nx, ny = 130, 77
    if kw.pop("obstacles", False):
        kw["obstacles"] = _mask(nx, ny, 5)
    gpu, ora = make_pair(nx, ny, storage=storage, init=random_fields(nx, ny, 7, du=0.02),
                         collision="trt", magic=magic, **kw)
    for n in (1, 9, 150):
        gpu.step(n)
        ora.run(n)
        drho, err = velocity_error(gpu, ora)
        emax = velocity_max_error(gpu, ora)
        print(f"TRT {case} magic {magic:.4f} {storage} step {gpu.time}: drho {drho:.2e} "
              f"err {err:.2e} max {emax:.2e}")
        assert err < tol and emax < 10 * tol, (n, drho, err, emax)
    gpu.close()


def test_trt_with_a_moving_disc_against_oracle():
    nx, ny = 96, 64
    gpu, ora = make_pair(nx, ny, storage="f64", bc_y="wall", tau=0.75, g=(2e-6, 0.0),
                         particles=[dict(x=40.3, y=31.7, radius=6.0, density_ratio=1.2)],
                         collision="trt", magic=0.25)
    gpu.step(200)
    ora.run(200)
    _, err = velocity_error(gpu, ora)
    pg, po = gpu.particles(), ora.particles()
    dstate = np.abs(pg[:, :7] - po[:, :7]).max()
    print(f"TRT disc f64: velocity err {err:.2e}, particle state {dstate:.2e}")
    assert err < 1e-11 and dstate < 1e-11
    gpu.close()


FORMATS = [("f64", "nearest"), ("f32", "nearest"), ("f32", "stochastic"), ("f16", "stochastic"),
           ("bf16", "stochastic")]


@pytest.mark.parametrize("storage,rounding", FORMATS)
@pytest.mark.parametrize("power_law", [None, 0.5])
def test_trt_two_step_equals_single_steps(storage, rounding, power_law):
    pl = None if power_law is None else dict(n=power_law, K=0.01, tau_min=0.51, tau_max=2.5)
    for (nx, ny), kw in (((130, 77), dict(obstacles=_mask(130, 77, 3))), ((64, 40), dict(bc_y="wall"))):
        out = []
        for two in (1, 0):
            d = lb.Domain(nx, ny, tau=0.7, g=(3e-6, 1e-6), storage=storage, rounding=rounding,
                          power_law=pl, init=random_fields(nx, ny, 4, du=0.02), seed=5, domain_id=2,
                          collision="trt", magic=0.3, **kw)
            d.set_option(lb.OPT_TWO_STEP, two)
            d.step(27)
            out.append(d.populations())
            d.close()
        assert np.array_equal(out[0], out[1]), (storage, rounding, power_law, nx, ny)


def test_trt_poiseuille_walls_exactly_halfway():
    """FP64, magic 3/16: the steady channel profile is the parabola with the
    walls halfway between the solid and the first fluid row, for tau 0.9 and
    1.8 (BGK at 1.8 slips by about 1 % of the peak)."""
    ny, g = 34, 1e-6
    y = np.arange(1, ny - 1)
    for tau in (0.9, 1.8):
        d = lb.Domain(64, ny, tau=tau, g=(g, 0.0), bc_y="wall", storage="f64", collision="trt",
                      magic=3.0 / 16.0)
        d.step(30000)
        _, u, _ = d.moments()
        nu = (tau - 0.5) / 3
        parabola = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
        dev = np.abs(u[1:-1] - parabola[:, None]).max() / parabola.max()
        print(f"TRT plane Poiseuille tau {tau}: max deviation from the parabola {dev:.2e}")
        assert dev < 1e-10
        d.close()
