"""The Brownian disc of the fluctuating workload (Sec. 4: a disc of radius 5
in a 512^2 periodic fluid at kT = 1e-4, tau = 1): its mean-squared
displacement over 1e5 steps, ballistic at short lags and diffusive at long
ones, against the regression of fluctuations (Onsager): the velocity
autocorrelation decays as the disc's deterministic response to an impulse,
C(t) = <U_x^2> R(t), so MSD(t) = 4 int_0^t (t - s) C(s) ds.  R(t) comes from
a noise-free run of the same lattice; <U_x^2> and the MSD from 16 seeded
realisations batched in one launch, time-averaged over their trajectories.
The periodic-array drag (Hasimoto; Sangani & Acrivos) gives the long-time
diffusion coefficient D = kT / zeta of a disc in this box, approached only for
lags beyond L^2 / nu ~ 1.6e6 steps (the 2D velocity autocorrelation decays as
1/t), so the measured MSD / 4t at lag 5000 is checked against it loosely."""
import numpy as np
import pytest

import closed_forms as cf

pytestmark = pytest.mark.gpu

N, R, KT, TAU = 512, 5.0, 1e-4, 1.0
SAMPLE = 10          # steps between recorded positions
LAGS = (50, 500, 5000)


def _response(tmax):
    """Normalised velocity response R(t) = U_x(t) / U_x(0) of the disc to an
    impulse (initial velocity, fluid at rest), noise off, every step."""
    from paper_2006_12910_amd import lb
    d = lb.Domain(N, N, tau=TAU, storage="f64", max_particles=1)
    u0 = 1e-3
    d.add_particles([dict(x=N / 2 + 0.5, y=N / 2 + 0.5, radius=R, ux=u0)])
    out = [1.0]
    for t in range(tmax):
        d.step(1)
        out.append(d.particles()[0][4] / u0)
    d.close()
    return np.array(out)


def _msd_prediction(c0, resp, lag):
    """4 int_0^lag (lag - s) c0 R(s) ds (trapezoid on the unit step grid);
    the disc moves by its velocity before the update, x(t+1) = x(t) + U(t),
    so the sum form is used: 2 sum_{i,j<lag} C(|i - j|) per component."""
    c = c0 * resp[:lag]
    k = np.arange(lag)
    per_component = lag * c[0] + 2.0 * ((lag - k[1:]) * c[1:]).sum()
    return 2.0 * per_component


def test_brownian_disc_msd_follows_the_regression_of_fluctuations():
    from paper_2006_12910_amd import lb
    resp = _response(max(LAGS))
    members = 16
    doms = []
    for k in range(members):
        d = lb.Domain(N, N, tau=TAU, storage="f32", kT=KT, seed=2006, domain_id=100 + k,
                      max_particles=1)
        d.add_particles([dict(x=N / 2 + 0.5, y=N / 2 + 0.5, radius=R)])
        doms.append(d)
    batch = lb.Batch(doms)
    batch.step(5000)  # the fluid modes that set the lags below thermalise
    steps = 100000
    nrec = steps // SAMPLE
    pos = np.zeros((members, nrec + 1, 2))
    vel = np.zeros((members, nrec + 1, 2))
    last = np.array([d.particles()[0][0:2] for d in doms])
    for k in range(nrec + 1):
        if k:
            batch.step(SAMPLE)
        if k % 2000 == 0:
            print(f"brownian ensemble: step {doms[0].time}", flush=True)
        p = np.array([d.particles()[0] for d in doms])
        step = p[:, 0:2] - last  # unwrap across the periodic edges
        step -= N * np.round(step / N)
        pos[:, k] = (pos[:, k - 1] if k else 0.0) + step
        vel[:, k] = p[:, 4:6]
        last = p[:, 0:2]
    batch.close()
    for d in doms:
        d.close()
    c0 = (vel ** 2).mean() / 1.0  # <U_x^2> = <U_y^2>: per component
    m = np.pi * R * R
    # sampling error from the spread of the 16 independent realisations
    per_member = m * (vel ** 2).mean(axis=(1, 2)) / KT
    se = per_member.std(ddof=1) / np.sqrt(members)
    print(f"disc translation energy m <U_x^2> / kT = {m * c0 / KT:.3f} +- {se:.3f} (16 realisations)")
    # the disc runs ~10 % hot (measured 1.10-1.13, far outside the sampling
    # error): a systematic excess of the particle coupling, not of the noise,
    # whose fluid equipartition holds to 0.2 %
    assert se < 0.05
    assert 0.95 < m * c0 / KT < 1.25
    D_per = KT * (-0.5 * np.log(np.pi * R * R / N ** 2) - 0.738 + np.pi * R * R / N ** 2) / (
        4 * np.pi * cf.nu_of_tau(TAU))
    for lag in LAGS:
        j = lag // SAMPLE
        d2 = ((pos[:, j:] - pos[:, :-j]) ** 2).sum(-1).mean()
        pred = _msd_prediction(c0, resp, lag)
        print(f"lag {lag}: MSD {d2:.4e}, regression {pred:.4e} (ratio {d2 / pred:.3f}), "
              f"MSD/4t {d2 / (4 * lag):.3e} (periodic-array D {D_per:.3e})")
        assert abs(d2 / pred - 1) < (0.1 if lag < 5000 else 0.2), (lag, d2, pred)
    # diffusive at long lags: between the crossover and the periodic limit
    assert 0.3 < (d2 / (4 * LAGS[-1])) / D_per < 1.3
