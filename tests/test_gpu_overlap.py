"""Overlapped particle steps (LB_OPT_OVERLAP): the particle coupling and the
sweep of the tiles within its reach run on a second stream beside the sweep of
the other tiles.  The populations, particle states and labels must equal the
serial order bit for bit: with obstacles and walls, with particles that cross
a periodic edge, in every storage format, replayed from graphs and eager."""
import numpy as np
import pytest

from paper_2006_12910_amd import inputs, lb

pytestmark = pytest.mark.gpu


def _domain(case, storage, overlap, use_graph):
    if case == "porous":
        nx, ny = 320, 160
        mask, _ = inputs.rsa_discs(nx, ny, 4.0, 9.0, 0.12, 1.0, inputs.rng(8), periodic=False)
        mask[:, :40] = 0  # room for the particles
        mask[0, :] = mask[-1, :] = 1
        parts = [dict(x=12.5, y=40.5, radius=6.0, density_ratio=1.2, ux=0.02),
                 dict(x=20.0, y=80.0, radius=7.5, density_ratio=1.5, uy=0.01, omega=0.001),
                 dict(x=14.0, y=118.0, radius=5.0, density_ratio=1.1)]
        d = lb.Domain(nx, ny, tau=0.7, g=(3e-5, 0.0), bc_x="periodic", bc_y="wall", storage=storage,
                      rounding="stochastic" if storage in ("f16", "bf16") else "nearest",
                      obstacles=mask, max_particles=4, lj=(1e-3, 2.5, 0.5), seed=3)
    else:  # periodic box, particles across both periodic edges
        nx, ny = 200, 136
        parts = [dict(x=2.0, y=60.0, radius=6.0, density_ratio=1.3, ux=-0.02),
                 dict(x=100.0, y=134.0, radius=7.0, density_ratio=1.4, uy=0.015),
                 dict(x=197.5, y=1.5, radius=5.5, density_ratio=1.2, ux=0.01, uy=-0.01)]
        d = lb.Domain(nx, ny, tau=0.8, g=(1e-5, 2e-6), storage=storage,
                      rounding="stochastic" if storage in ("f16", "bf16") else "nearest",
                      max_particles=3, lj=(1e-3, 2.5, 0.5), seed=4)
    d.set_option(lb.OPT_OVERLAP, overlap)
    d.set_option(lb.OPT_USE_GRAPH, use_graph)
    d.add_particles(parts)
    return d


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", ["porous", "periodic"])
def test_overlapped_steps_equal_serial(case, storage):
    for use_graph in (1, 0):
        a = _domain(case, storage, 1, use_graph)
        b = _domain(case, storage, 0, use_graph)
        assert a.get_option(lb.OPT_OVERLAP) == 1
        for n in (1, 6, 33):  # calls of several lengths: the call boundary too
            a.step(n)
            b.step(n)
        assert a.time == b.time == 40
        assert np.array_equal(a.particles(), b.particles())
        assert np.array_equal(a.populations(), b.populations())
        ra, rb = a.moments(), b.moments()
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y)
        assert a.mass() == b.mass()
        a.close()
        b.close()


def test_overlap_option_values():
    d = _domain("periodic", "f32", 0, 1)
    assert d.get_option(lb.OPT_OVERLAP) == 0
    with pytest.raises(lb.LBError):
        d.set_option(lb.OPT_OVERLAP, 2)
    d.close()


def test_overlapped_steps_match_the_oracle():
    """FP64 storage: the overlapped order against the FP64 oracle (walls,
    obstacles, three moving particles)."""
    from helpers import make_pair, velocity_error
    nx, ny = 320, 160
    mask, _ = inputs.rsa_discs(nx, ny, 4.0, 9.0, 0.12, 1.0, inputs.rng(8), periodic=False)
    mask[:, :40] = 0
    mask[0, :] = mask[-1, :] = 1
    parts = [dict(x=12.5, y=40.5, radius=6.0, density_ratio=1.2, ux=0.02),
             dict(x=20.0, y=80.0, radius=7.5, density_ratio=1.5, uy=0.01, omega=0.001),
             dict(x=14.0, y=118.0, radius=5.0, density_ratio=1.1)]
    gpu, ora = make_pair(nx, ny, tau=0.7, g=(3e-5, 0.0), obstacles=mask, particles=parts,
                         lj=(1e-3, 2.5, 0.5), max_particles=4)
    gpu.set_option(lb.OPT_OVERLAP, 1)
    for n in (1, 6, 33):
        gpu.step(n)
        ora.run(n)
        drho, err = velocity_error(gpu, ora)
        pd = np.abs(gpu.particles()[:, :7] - ora.particles()[:, :7]).max()
        assert drho < 1e-13 and err < 1e-11 and pd < 1e-13, (n, drho, err, pd)
    gpu.close()
