"""Properties of the seeded stand-ins for the paper's timing benchmarks (no
lattice-Boltzmann arithmetic is involved: these are the inputs both sides of a
parity check start from)."""
import itertools

import numpy as np

from paper_2006_12910_amd import inputs


def test_replica_b1_layout():
    """Sec. 6, first benchmark: 1020 x 1620 lattice, 45 particles of radius
    6.5 with surface spacings 8.5 and 5.5, released into a grain-free band of
    a disordered porous medium between lateral walls."""
    mask, centres = inputs.replica_b1()
    ny, nx = mask.shape
    assert (nx, ny) == (1020, 1620)
    assert len(centres) == 45
    assert abs(mask.mean() - 0.30) < 0.01
    assert mask[ny - 220:].sum() == 0  # release band is grain-free
    r = 6.5
    ys, xs = np.mgrid[0:ny, 0:nx]
    for cx, cy in centres:
        # no node on a surface, no grain or wall node inside a particle
        inside = (xs - cx) ** 2 + (ys - cy) ** 2 < r * r
        assert not np.any(np.isclose((xs - cx) ** 2 + (ys - cy) ** 2, r * r))
        assert mask[inside].sum() == 0
        assert cx - r > 1 and cx + r < nx - 2
    gaps = [np.hypot(a[0] - b[0], a[1] - b[1]) - 2 * r for a, b in itertools.combinations(centres, 2)]
    assert min(gaps) >= 5.5 - 1e-9
    row = sorted(c for c in centres if c[1] == centres[0][1])
    assert np.allclose(np.diff([c[0] for c in row]), 2 * r + 8.5)


def test_replica_b2_disc_sits_in_the_channel():
    """Sec. 6, second benchmark: 3000 x 41 channel, one disc of radius 7.5."""
    ((cx, cy),) = inputs.replica_b2()
    r = 7.5
    assert r + 2 < cy < 40 - r - 2 and 0 < cx < 3000
    ys, xs = np.mgrid[0:41, int(cx) - 10:int(cx) + 11]
    assert not np.any(np.isclose((xs - cx) ** 2 + (ys - cy) ** 2, r * r))
