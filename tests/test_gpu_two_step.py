"""The two-step sweep (two time steps per pass over memory, first step held in
on-chip memory) against single steps: the stored populations must be
bit-identical, for every storage format and rounding, with and without
obstacles, on ragged lattice sizes (narrower than one tile too), for step
counts with and without a remainder, alone and batched."""
import numpy as np
import pytest

from paper_2006_12910_amd import inputs, lb

pytestmark = pytest.mark.gpu

FORMATS = [("f64", "nearest"), ("f32", "nearest"), ("f32", "stochastic"), ("f16", "stochastic"),
           ("f16", "nearest"), ("bf16", "stochastic")]
SHAPES = [(130, 77), (64, 64), (300, 33), (40, 50)]


def _fields(nx, ny, seed):
    r = np.random.default_rng(seed)
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    ux = 0.02 * np.sin(2 * np.pi * y / ny + 0.4) + 0.003 * r.standard_normal((ny, nx))
    uy = 0.01 * np.cos(2 * np.pi * x / nx) + 0.003 * r.standard_normal((ny, nx))
    return 1.0 + 0.004 * r.standard_normal((ny, nx)), ux, uy


def _mask(nx, ny, seed):
    m, _ = inputs.rsa_discs(nx, ny, 3.0, 7.0, 0.2, 1.0, inputs.rng(seed), periodic=True)
    return m


def _domain(nx, ny, storage, rounding, obstacles, two, seed=3):
    d = lb.Domain(nx, ny, tau=0.62, g=(2e-6, -1e-6), storage=storage, rounding=rounding,
                  obstacles=_mask(nx, ny, seed) if obstacles else None, init=_fields(nx, ny, seed),
                  seed=77, domain_id=seed)
    d.set_option(lb.OPT_TWO_STEP, two)
    return d


@pytest.mark.parametrize("storage,rounding", FORMATS)
@pytest.mark.parametrize("obstacles", [False, True])
def test_two_step_equals_single_steps(storage, rounding, obstacles):
    for nx, ny in SHAPES:
        for steps in (4, 7, 261):
            a = _domain(nx, ny, storage, rounding, obstacles, 1)
            b = _domain(nx, ny, storage, rounding, obstacles, 0)
            a.step(steps)
            b.step(steps)
            fa, fb = a.populations(), b.populations()
            assert a.time == b.time == steps
            assert np.array_equal(fa, fb), (nx, ny, steps, np.abs(fa - fb).max())
            a.close()
            b.close()


HEIGHTS = {"f64": (4, 6, 8), "f32": (6, 10, 14), "f16": (10, 14, 18), "bf16": (10, 14, 18)}


@pytest.mark.parametrize("storage,rounding", FORMATS)
def test_every_tile_height_equals_single_steps(storage, rounding):
    """Each instantiated two-step tile height (LB_OPT_TWO_STEP_ROWS) gives
    the single-step result bit for bit."""
    for nx, ny in ((130, 77), (300, 33)):
        b = _domain(nx, ny, storage, rounding, True, 0)
        b.step(23)
        ref = b.populations()
        b.close()
        for h in HEIGHTS[storage]:
            a = _domain(nx, ny, storage, rounding, True, 1)
            a.set_option(lb.OPT_TWO_STEP_ROWS, h)
            assert a.get_option(lb.OPT_TWO_STEP_ROWS) == h
            a.step(23)
            assert np.array_equal(a.populations(), ref), (storage, nx, ny, h)
            a.close()
    d = _domain(64, 64, storage, rounding, False, 1)
    with pytest.raises(lb.LBError):
        d.set_option(lb.OPT_TWO_STEP_ROWS, 12)
    d.close()


def test_batch_tile_height_and_autotune():
    """The batch's own tile height (option and autotuner, with its cache):
    the members still evolve exactly as under single steps."""
    shapes = [(130, 77, False), (64, 64, True), (300, 33, True), (257, 129, True)]
    ref = None
    for mode in ("single", "rows10", "tuned", "tuned-again"):
        doms = [_domain(nx, ny, "f16", "stochastic", obs, 0 if mode == "single" else 1, seed=20 + i)
                for i, (nx, ny, obs) in enumerate(shapes)]
        batch = lb.Batch(doms)
        if mode == "rows10":
            batch.set_option(lb.OPT_TWO_STEP_ROWS, 10)
        elif mode.startswith("tuned"):
            ms = batch.autotune(steps=8)
            assert ms >= 0 and (mode == "tuned" or ms == 0)  # the second time from the cache
        done = doms[0].time
        batch.step(64 - done)
        pops = [d.populations() for d in doms]
        if ref is None:
            ref = pops
        else:
            for f, g in zip(pops, ref):
                assert np.array_equal(f, g), mode
        with pytest.raises(lb.LBError):
            batch.set_option(lb.OPT_TWO_STEP_ROWS, 7)
        batch.close()
        for d in doms:
            d.close()


def test_two_step_batch_equals_single_steps():
    shapes = [(130, 77, False), (64, 64, True), (300, 33, True), (40, 50, False), (257, 129, True)]
    for two in (1, 0):
        doms = [_domain(nx, ny, "f16", "stochastic", obs, two, seed=10 + i)
                for i, (nx, ny, obs) in enumerate(shapes)]
        batch = lb.Batch(doms)
        batch.step(259)
        if two:
            ref = [d.populations() for d in doms]
        else:
            for d, f in zip(doms, ref):
                assert np.array_equal(d.populations(), f)
        batch.close()
        for d in doms:
            d.close()


@pytest.mark.parametrize("storage,rounding", FORMATS)
@pytest.mark.parametrize("power_law", [None, 0.5, 0.75, 1.5, 1.3])
def test_two_step_with_walls_and_power_law_equals_single_steps(storage, rounding, power_law):
    """Channels: walls held as solid label rows (walls in y, and in x too),
    Newtonian or with the power-law relaxation time (every closed-form
    specialisation and the generic Newton solve): two-step launches equal
    single steps bit for bit."""
    pl = None if power_law is None else dict(n=power_law, K=0.01, tau_min=0.51, tau_max=2.5)
    for (nx, ny), walls in (((130, 77), dict(bc_y="wall")), ((64, 40), dict(bc_x="wall", bc_y="wall"))):
        out = []
        for two in (1, 0):
            d = lb.Domain(nx, ny, tau=0.7, g=(3e-6, 0.0), storage=storage, rounding=rounding,
                          power_law=pl, init=_fields(nx, ny, 9), seed=5, domain_id=2, **walls)
            d.set_option(lb.OPT_TWO_STEP, two)
            d.step(27)
            out.append(d.populations())
            d.close()
        assert np.array_equal(out[0], out[1]), (storage, rounding, power_law, nx, ny)


def test_two_step_not_taken_where_not_supported():
    """Pressure faces, particles or noise keep single steps: the option is
    accepted and the results still equal the single-step ones."""
    for kw in (dict(bc_x="pressure", bc_y="wall", rho_in=1.001, rho_out=0.999), dict(kT=1e-5)):
        doms = []
        for two in (1, 0):
            d = lb.Domain(96, 40, tau=0.8, storage="f32", init=_fields(96, 40, 5), **kw)
            d.set_option(lb.OPT_TWO_STEP, two)
            d.step(9)
            doms.append(d)
        assert np.array_equal(doms[0].populations(), doms[1].populations())
        for d in doms:
            d.close()


def test_autotune_times_single_steps_and_keeps_the_option():
    """The autotuner tunes the single-step tiles with the two-step sweep off,
    then restores it; the steps it timed advance the state exactly as plain
    steps do (tiles do not change results)."""
    a = _domain(300, 140, "f16", "stochastic", True, 1)
    b = _domain(300, 140, "f16", "stochastic", True, 1)
    ms = a.autotune(steps=4)
    assert ms > 0
    assert a.get_option(lb.OPT_TWO_STEP) == 1
    assert a.get_option(lb.OPT_TILE_WIDTH) in (64, 128, 256)
    assert a.get_option(lb.OPT_ROWS_PER_THREAD) in (2, 4, 8)
    assert a.get_option(lb.OPT_TWO_STEP_ROWS) in HEIGHTS["f16"]
    t = a.time
    assert t > 0 and t % 8 == 0  # warm-up and timed runs of 4 steps per shape
    b.step(t)
    a.step(6)
    b.step(6)
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()
