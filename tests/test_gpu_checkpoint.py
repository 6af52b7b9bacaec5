"""Checkpoint and resume (the paper's dumps for restarts, Sec. 7): a fresh
domain given the step count, the populations and the particle state of a
checkpoint continues bit for bit as the original, with noise, obstacles,
walls, moving particles crossing nodes and the two-step force mean."""
import numpy as np
import pytest

from paper_2006_12910_amd import inputs, lb

pytestmark = pytest.mark.gpu


def _mask(nx, ny):
    m, _ = inputs.rsa_discs(nx, ny, 4.0, 8.0, 0.10, 1.5, inputs.rng(31), periodic=False)
    m[:, :60] = 0
    return m


def _domain(storage, rounding, mask, parts):
    d = lb.Domain(180, 96, tau=0.75, g=(2e-5, -3e-6), bc_y="wall", storage=storage,
                  rounding=rounding, kT=2e-5, seed=99, domain_id=4, obstacles=mask,
                  max_particles=4, lj=(1e-3, 2.5, 0.5))
    d.set_option(lb.OPT_FORCE_AVERAGE, 1)
    if parts:
        d.add_particles(parts)
    return d


PARTS = [dict(x=14.5, y=30.5, radius=6.0, density_ratio=1.3, ux=0.03, uy=0.004),
         dict(x=30.2, y=62.7, radius=7.0, density_ratio=1.1, ux=0.02, omega=0.002),
         dict(x=45.0, y=20.0, radius=5.0, density_ratio=2.0, ux=0.01, uy=0.01)]


@pytest.mark.parametrize("storage,rounding", [("f64", "nearest"), ("f32", "stochastic"),
                                              ("f16", "stochastic")])
def test_resume_from_checkpoint_is_bit_exact(storage, rounding):
    mask = _mask(180, 96)
    a = _domain(storage, rounding, mask, PARTS)
    a.step(37)  # odd: the resumed domain's state moves to the other buffer
    t = a.time
    f = a.populations()
    ps = a.particle_state()
    assert np.abs([ps[0][k].cover_fx for k in range(3)]).max() >= 0  # readable
    a.step(41)

    b = _domain(storage, rounding, mask, [])
    b.set_time(t)
    b.set_populations(f)
    b.set_particle_state(ps)
    assert b.time == t and b.num_particles == 3
    b.step(41)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.particles(), b.particles())
    ra, rb = a.moments(), b.moments()
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_particle_state_replaces_particles_and_relabels():
    """Setting a state with the particles elsewhere clears the old particle
    labels: the run equals one that started with the new state."""
    mask = _mask(180, 96)
    src = _domain("f64", "nearest", mask, PARTS)
    src.step(20)
    ps = src.particle_state()
    f = src.populations()
    moved = _domain("f64", "nearest", mask, [dict(x=120.5, y=50.5, radius=6.0)])
    moved.step(20)  # same step count, particle elsewhere
    moved.set_populations(f)
    moved.set_particle_state(ps)
    src.step(15)
    moved.step(15)
    assert np.array_equal(src.populations(), moved.populations())
    assert np.array_equal(src.particles(), moved.particles())
    empty = (lb.ParticleState * 1)()
    moved.set_particle_state((empty, 0))
    assert moved.num_particles == 0
    moved.step(2)
    src.close()
    moved.close()


def test_set_particle_state_rejects_bad_states():
    mask = _mask(180, 96)
    d = _domain("f64", "nearest", mask, PARTS)
    arr, n = d.particle_state()
    solid = np.argwhere(mask)[0]
    arr[0].p.x, arr[0].p.y = float(solid[1]), float(solid[0])
    with pytest.raises(lb.LBError) as e:
        d.set_particle_state((arr, n))
    assert e.value.status == lb.LB_EINVAL
    arr, n = d.particle_state()
    arr[1].cover_fx = float("nan")
    with pytest.raises(lb.LBError):
        d.set_particle_state((arr, n))
    with pytest.raises(lb.LBError):
        d.set_time(-1)
    d.close()
