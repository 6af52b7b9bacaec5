"""Pins of the oracle's fluctuating LB (Sec. 4): equipartition of the velocity
and density fluctuations, which linear fluctuating-hydrodynamics theory makes
exact for a noise that obeys the fluctuation-dissipation theorem."""
import numpy as np
import pytest

from oracle import Oracle, OracleParams


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_equipartition(tau):
    kT = 1e-4
    o = Oracle(OracleParams(nx=32, ny=32, tau=tau, kT=kT, seed=77)).run(500)
    a, b, c = [], [], []
    for _ in range(3000):
        o.run(1)
        r, ux, uy = o.moments()
        a.append((r * ux * ux).mean())
        b.append((r * uy * uy).mean())
        c.append(((r - 1) ** 2).mean())
    assert abs(np.mean(a) / kT - 1) < 0.02
    assert abs(np.mean(b) / kT - 1) < 0.02
    assert abs(np.mean(c) / (3 * kT) - 1) < 0.02


def test_noise_is_deterministic_per_seed_and_domain():
    def run(seed, dom):
        return Oracle(OracleParams(nx=12, ny=10, tau=0.9, kT=1e-4, seed=seed,
                                   domain_id=dom)).run(4).populations()
    a = run(1, 0)
    assert np.array_equal(a, run(1, 0))
    assert not np.array_equal(a, run(2, 0))
    assert not np.array_equal(a, run(1, 1))
