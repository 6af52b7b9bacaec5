"""Parity and invariants at the full sizes of the five benchmark workloads,
in the launch configuration the benchmark uses (graph-captured steps).

Where the oracle can follow the full lattice for a bounded number of steps it
does (FP64 storage to accumulated rounding, FP32 to the 1e-5 target); for the
long runs the checks are properties that hold at any size: x-invariance of a
channel flow started x-uniform, the closed-form power-law profile, the
closed-form decay of a shear wave, equipartition of thermal fluctuations,
FP32 against FP64 runs of the same lattice, and batched against solo runs.
"""
import numpy as np
import pytest

from helpers import make_pair, rel_l2, velocity_error, velocity_max_error
import closed_forms as cf

pytestmark = pytest.mark.gpu


def _particle_state_diff(gpu, ora):
    pg, po = gpu.particles(), ora.particles()
    return np.abs(pg[:, :7] - po[:, :7]).max()


# --- porous flow with mobile particles: 2048 x 1024, 35 % discs, 16 discs R = 8
#
# Repulsion (Eq. MP2) with r_it = 2.5 and psi = 1e-3 in lattice units.  The
# paper's psi = 20 is not in lattice units: at the threshold it accelerates an
# R = 8 disc (m = 1.05 pi 64 = 211) by 0.1 node/step^2 and the explicit
# Newton-Euler step diverges within steps of the first contact.  psi = 1e-3
# is of the order of the hydrodynamic force on a disc here (the pressure
# gradient 3.3e-7 over 200 node^2 gives 7e-5), so contacts stay gentle.
# The particle update takes the mean of two steps' forces: with the explicit
# update of Eq. MP5 the near-neutral discs of the block start a period-two
# oscillation that grows without bound after ~2000 steps.
_LJ = (1e-3, 2.5, 0.5)


def _porous(storage, compute="native"):
    from paper_2006_12910_amd import inputs
    mask, _ = inputs.porous_channel()
    parts = [dict(x=x, y=y, radius=8.0, density_ratio=1.05) for x, y in inputs.particle_block()]
    return make_pair(2048, 1024, storage=storage, compute=compute, bc_x="pressure", bc_y="wall",
                     tau=0.7, rho_in=1.001, rho_out=0.999, obstacles=mask, particles=parts, lj=_LJ,
                     force_average=True)


@pytest.mark.parametrize("storage,compute,tol,ptol", [("f64", "native", 1e-10, 1e-11),
                                                      ("f32", "f64", 1e-5, 1e-6),
                                                      ("f32", "native", 1e-5, 1e-5)])
def test_porous_full_lattice_against_oracle(storage, compute, tol, ptol):
    """FP32 storage meets the 1e-5 target with FP32 and with FP64 arithmetic.
    The density faces hold rho_in - rho0 = 1e-3 as one FP32 number (the
    difference of the two FP32-rounded densities erred by 5e-5 of it)."""
    gpu, ora = _porous(storage, compute)
    gpu.step(200)
    ora.run(200)
    drho, err = velocity_error(gpu, ora)
    emax = velocity_max_error(gpu, ora)
    state = _particle_state_diff(gpu, ora)
    print(f"porous {storage}/{compute}: drho {drho:.2e} err {err:.2e} max {emax:.2e} "
          f"particle state {state:.2e}")
    assert err < tol and emax < tol, (err, emax)
    assert state < ptol, state


def test_porous_20000_steps_fluid_fp32_tracks_fp64():
    """The full run length without the particles: FP32 storage (FP64
    arithmetic) against FP64 storage to the FP32 target."""
    from paper_2006_12910_amd import inputs, lb
    mask, _ = inputs.porous_channel()
    kw = dict(bc_x="pressure", bc_y="wall", tau=0.7, rho_in=1.001, rho_out=0.999, obstacles=mask)
    a = lb.Domain(2048, 1024, storage="f64", **kw)
    b = lb.Domain(2048, 1024, storage="f32", compute="f64", **kw)
    for k in range(4):
        a.step(5000)
        b.step(5000)
        print(f"porous fluid: step {a.time}, mass {a.mass():.9f}", flush=True)
    _, ua, va = a.moments()
    _, ub, vb = b.moments()
    err = np.sqrt(((ua - ub) ** 2 + (va - vb) ** 2).sum() / (ua ** 2 + va ** 2).sum())
    print(f"porous fluid 20000 steps: f32 vs f64 velocity {err:.2e}, |u| max {np.hypot(ua, va).max():.2e}")
    assert err < 1e-5, err


def _inside_discs(p, nx, ny):
    yy, xx = np.mgrid[0:ny, 0:nx]
    inside = np.zeros((ny, nx), bool)
    for k in range(p.shape[0]):
        inside |= (xx - p[k, 0]) ** 2 + (yy - p[k, 1]) ** 2 < p[k, 2] ** 2
    return inside


def test_porous_20000_steps_with_particles_stays_physical():
    """The full run with the 16 discs (FP32 storage, FP64 arithmetic): the
    fluid outside and inside the discs stays finite, near rho0 and slow, the
    discs stay slow and clear of the obstacles and of each other, and they
    are carried downstream.  The fluid inside a disc meets the outside only
    through the covered/uncovered nodes (the link force of Eq. MP1 is taken
    on the exterior side), so it is checked on its own."""
    from paper_2006_12910_amd import inputs
    g, _ = _porous("f32", "f64")
    p0 = g.particles().copy()
    for k in range(10):
        g.step(2000)
        p = g.particles()
        print(f"porous particles: step {g.time}, max |U| {np.abs(p[:, 4:6]).max():.2e}", flush=True)
    r, u, v = g.moments()
    ext = (r > 0) & ~_inside_discs(p, 2048, 1024)
    inn = (r > 0) & ~ext
    speed = np.hypot(u, v)
    print(f"exterior rho in [{r[ext].min():.5f}, {r[ext].max():.5f}], |u| max {speed[ext].max():.2e}; "
          f"interior rho in [{r[inn].min():.5f}, {r[inn].max():.5f}], |u| max {speed[inn].max():.2e}")
    assert np.isfinite(r).all() and 0.998 < r[ext].min() and r[ext].max() < 1.002
    assert speed[ext].max() < 0.005
    assert 0.995 < r[inn].min() and r[inn].max() < 1.005 and speed[inn].max() < 0.005
    mask, _ = inputs.porous_channel()
    sy, sx = np.nonzero(mask)
    for k in range(p.shape[0]):
        x, y, rad = p[k, 0], p[k, 1], 8.0
        assert 0 < x < 2048 and rad < y < 1023 - rad
        assert np.sqrt((sx - x) ** 2 + (sy - y) ** 2).min() > rad - 1.0, k
        for j in range(k):
            assert np.hypot(p[j, 0] - x, p[j, 1] - y) > 2 * rad - 1.0, (j, k)
    assert (p[:, 0] > p0[:, 0]).mean() > 0.5  # downstream on the whole
    assert np.abs(p[:, 4:6]).max() < 0.005


# --- fluctuating fluid with a Brownian disc: 512^2, kT = 1e-4, tau = 1

def _fluct(storage, n=512, seed=2006, domain_id=1):
    return make_pair(n, n, storage=storage, tau=1.0, kT=1e-4, seed=seed, domain_id=domain_id,
                     particles=[dict(x=n / 2 + 0.5, y=n / 2 + 0.5, radius=5.0)])


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_fluctuating_full_lattice_against_oracle(storage, tol):
    gpu, ora = _fluct(storage)
    gpu.step(100)
    ora.run(100)
    drho, err = velocity_error(gpu, ora)
    emax = velocity_max_error(gpu, ora)
    state = _particle_state_diff(gpu, ora)
    print(f"fluctuating {storage}: drho {drho:.2e} err {err:.2e} max {emax:.2e} "
          f"particle state {state:.2e}")
    assert err < tol and emax < tol and state < (1e-11 if storage == "f64" else 1e-6), (err, state)


def test_fluctuating_100000_steps_equipartition():
    """Over the full run: the fluid velocity and density variances equal kT
    and 3 kT (linear fluctuating hydrodynamics with a noise obeying the
    fluctuation-dissipation theorem); the disc's kinetic energy per degree
    of freedom is kT within the sampling error of its correlated samples."""
    from paper_2006_12910_amd import lb
    kT = 1e-4
    gpu = lb.Domain(512, 512, tau=1.0, storage="f32", kT=kT, seed=2006, domain_id=1,
                    max_particles=1)
    gpu.add_particles([dict(x=256.5, y=256.5, radius=5.0)])
    gpu.step(20000)
    fu, fv, fr, pu, pw = [], [], [], [], []
    for k in range(800):
        if k % 100 == 0:
            print(f"equipartition run: step {gpu.time}", flush=True)
        gpu.step(100)
        p = gpu.particles()[0]
        pu.append(p[4:6].copy())
        pw.append(p[6])
        if k % 40 == 0:
            r, ux, uy = gpu.moments()
            fl = r > 0
            fu.append((r[fl] * ux[fl] ** 2).mean())
            fv.append((r[fl] * uy[fl] ** 2).mean())
            fr.append(((r[fl] - 1.0) ** 2).mean())
    assert gpu.time == 100000
    ex, ey, er = np.mean(fu) / kT, np.mean(fv) / kT, np.mean(fr) / (3 * kT)
    m = np.pi * 25.0  # rho_p = rho0 = 1
    inertia = 0.5 * m * 25.0
    pu = np.array(pu)
    et = m * (pu ** 2).mean() / kT
    erot = inertia * (np.array(pw) ** 2).mean() / kT
    print(f"equipartition: fluid u {ex:.4f} v {ey:.4f} rho {er:.4f}; disc translation {et:.3f} "
          f"rotation {erot:.3f}")
    assert abs(ex - 1) < 0.02 and abs(ey - 1) < 0.02 and abs(er - 1) < 0.02
    # one disc, 800 correlated samples: the disc's temperature is checked
    # loosely here (measured 1.10 / 1.22); the 16-realisation ensemble of the
    # MSD test bounds the translational one with its sampling error
    assert 0.9 < et < 1.35 and 0.9 < erot < 1.5


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_fluctuating_reduced_storage_equipartition(storage):
    """Thermal noise on 16-bit deviation storage with stochastic rounding
    (FP32 arithmetic): the fluid's velocity and density variances still
    equal kT and 3 kT (Eqs. NP1-NP2; linear fluctuating hydrodynamics).  The
    unbiased rounding adds a variance far below the noise's per step, so the
    bound is the sampling error of 200 snapshots of 256^2 nodes (~0.3 %)
    plus margin; round-to-nearest would damp or stall the fluctuations."""
    from paper_2006_12910_amd import lb
    kT, n = 1e-4, 256
    d = lb.Domain(n, n, tau=1.0, storage=storage, rounding="stochastic", kT=kT, seed=16,
                  domain_id=3)
    d.step(4000)
    fu, fv, fr = [], [], []
    for _ in range(200):
        d.step(50)
        r, ux, uy = d.moments()
        fu.append((r * ux ** 2).mean())
        fv.append((r * uy ** 2).mean())
        fr.append(((r - 1.0) ** 2).mean())
    ex, ey, er = np.mean(fu) / kT, np.mean(fv) / kT, np.mean(fr) / (3 * kT)
    print(f"{storage} equipartition: fluid u {ex:.4f} v {ey:.4f} rho {er:.4f}")
    assert abs(ex - 1) < 0.02 and abs(ey - 1) < 0.02 and abs(er - 1) < 0.02
    d.close()


def test_fluctuating_ensemble_batch():
    """64 realisations of 128^2..1024^2 in one batch: FP64 members match the
    oracle (the five smallest and the largest), FP32 members match their solo
    runs bit for bit."""
    from paper_2006_12910_amd import inputs, lb
    specs = inputs.fluctuating_batch(count=64)
    order = sorted(range(64), key=lambda i: specs[i]["n"])
    check = order[:5] + order[-1:]

    def member(spec, storage):
        n = spec["n"]
        cx, cy, r = spec["disc"]
        return make_pair(n, n, storage=storage, tau=1.0, kT=1e-4, seed=64, domain_id=spec["domain_id"],
                         particles=[dict(x=cx, y=cy, radius=r)])

    pairs = [member(s, "f64") for s in specs]
    batch = lb.Batch([g for g, _ in pairs])
    batch.step(30)
    for i in check:
        g, o = pairs[i]
        o.run(30)
        drho, err = velocity_error(g, o)
        assert drho < 1e-12 and err < 1e-10, (specs[i]["n"], drho, err)
    batch.close()
    for g, _ in pairs:
        g.close()
    del pairs

    grouped = [member(s, "f32")[0] for s in specs]
    batch = lb.Batch(grouped)
    batch.step(40)
    for i in check:
        solo = member(specs[i], "f32")[0]
        solo.step(40)
        assert np.array_equal(solo.populations(), grouped[i].populations()), specs[i]["n"]
        assert np.array_equal(solo.particles(), grouped[i].particles())
    batch.close()


# --- power-law channel: 4096 x 256, K = 0.01, tau* in [0.51, 2.5]

# body force per n giving a peak velocity of 0.05 (Mach 0.09) in the clamped
# closed form of the 254-node channel
_PL_G = {0.5: 2.7e-6, 0.75: 4e-7, 1.5: 2.07e-8}


def _pl_init(n, nx, ny):
    u = cf.powerlaw_channel(ny, n, 0.01, _PL_G[n], 0.51, 2.5)
    ux = np.zeros((ny, nx))
    ux[1:-1, :] = u[:, None]
    return np.ones((ny, nx)), ux, np.zeros((ny, nx)), u


@pytest.mark.parametrize("n", [0.5, 0.75, 1.5])
@pytest.mark.parametrize("storage,compute,rounding,tol", [("f64", "native", "nearest", 1e-10),
                                                          ("f32", "native", "stochastic", 1e-5),
                                                          ("f32", "native", "nearest", 2e-5),
                                                          ("f32", "f64", "nearest", 2e-5)])
def test_powerlaw_full_lattice_columns_match_oracle(n, storage, compute, rounding, tol):
    """Started x-uniform, every column of the full lattice equals the
    oracle's column of a narrow channel; with round-to-nearest storage the
    columns stay identical bit for bit (stochastic rounding draws different
    bits per node, so there each column is compared).

    FP32 storage meets the 1e-5 target with stochastic rounding.  With
    round-to-nearest storage the flow, started from its steady closed-form
    profile, changes by less per step than half the spacing of the stored
    FP32 values where tau* sits at its upper clamp (n = 0.5: the populations
    relax by 40 % of a tiny non-equilibrium part), so those values stagnate,
    in FP32 and FP64 arithmetic alike: bound 2e-5 (measured about 1.3e-5 for
    n = 0.5, below 2e-6 for the other two)."""
    from paper_2006_12910_amd import lb
    nx, ny = 4096, 256
    pl = dict(n=n, K=0.01, tau_min=0.51, tau_max=2.5)
    rho, ux, uy, _ = _pl_init(n, nx, ny)
    gpu = lb.Domain(nx, ny, storage=storage, compute=compute, rounding=rounding, bc_y="wall",
                    g=(_PL_G[n], 0.0), power_law=pl, init=(rho, ux, uy))
    _, ora = make_pair(4, ny, bc_y="wall", g=(_PL_G[n], 0.0), power_law=pl,
                       init=(rho[:, :4], ux[:, :4], uy[:, :4]))
    gpu.step(1500)
    ora.run(1500)
    rg, ug, vg = gpu.moments()
    ro, uo, vo = ora.moments()
    if rounding == "nearest":
        assert (ug == ug[:, :1]).all() and (vg == vg[:, :1]).all() and (rg == rg[:, :1]).all()
        err = rel_l2(ug[:, 0], uo[:, 0])
    else:
        cols = np.sqrt(((ug - uo[:, :1]) ** 2).sum(0) / (uo[:, 0] ** 2).sum())
        err = float(cols.max())
    print(f"power law n={n} {storage}/{compute}/{rounding}: column vs oracle {err:.2e}")
    assert err < tol, err


@pytest.mark.parametrize("n", [0.5, 0.75, 1.5])
@pytest.mark.parametrize("storage,rounding,tol", [("f64", "nearest", 1e-10),
                                                  ("f32", "stochastic", 1e-5)])
def test_powerlaw_full_lattice_perturbed_against_oracle(n, storage, rounding, tol):
    """The whole 4096 x 256 lattice started from the closed-form profile with
    a seeded perturbation that varies along x (a few long waves in both
    velocity components plus small random noise), so every column differs:
    the GPU against the oracle on the full lattice, node by node."""
    from paper_2006_12910_amd import lb
    nx, ny = 4096, 256
    pl = dict(n=n, K=0.01, tau_min=0.51, tau_max=2.5)
    rho, ux, uy, u = _pl_init(n, nx, ny)
    rng = np.random.default_rng(4096 + int(100 * n))
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    umax = np.abs(u).max()
    wall = np.zeros((ny, 1))
    wall[1:-1] = 1.0
    ux = ux * (1.0 + 0.05 * np.sin(2 * np.pi * 3 * x / nx)) + wall * 1e-3 * umax * rng.standard_normal((ny, nx))
    uy = wall * 0.02 * umax * np.sin(2 * np.pi * 5 * x / nx) * np.sin(np.pi * y / (ny - 1))
    rho = rho + wall * 1e-4 * np.cos(2 * np.pi * 2 * x / nx)
    gpu, ora = make_pair(nx, ny, storage=storage, rounding=rounding, bc_y="wall", g=(_PL_G[n], 0.0),
                         power_law=pl, init=(rho, ux, uy))
    gpu.step(300)
    ora.run(300)
    drho, err = velocity_error(gpu, ora)
    emax = velocity_max_error(gpu, ora)
    print(f"power law n={n} {storage}/{rounding} perturbed 4096x256: drho {drho:.2e} err {err:.2e} "
          f"max {emax:.2e}", flush=True)
    assert err < tol and emax < 10 * tol, (err, emax)


@pytest.mark.parametrize("n,tol", [(0.5, 2e-3), (0.75, 6e-4), (1.5, 1e-4)])
def test_powerlaw_full_lattice_holds_the_closed_form(n, tol):
    """FP32 storage with FP64 arithmetic: started from the clamped closed-form
    profile, 20000 steps later the profile still matches it (the discrete
    steady state differs from it by the lattice discretisation error) and no
    longer drifts."""
    from paper_2006_12910_amd import lb
    nx, ny = 4096, 256
    rho, ux, uy, ref = _pl_init(n, nx, ny)
    gpu = lb.Domain(nx, ny, storage="f32", compute="f64", bc_y="wall", g=(_PL_G[n], 0.0),
                    power_law=dict(n=n, K=0.01, tau_min=0.51, tau_max=2.5), init=(rho, ux, uy))
    gpu.step(10000)
    u1 = gpu.moments()[1][1:-1, 0].copy()
    gpu.step(10000)
    u2 = gpu.moments()[1][1:-1, 0]
    dev, drift = rel_l2(u2, ref), rel_l2(u2, u1)
    print(f"power law n={n}: vs closed form {dev:.2e}, drift over the last 10000 steps {drift:.2e}")
    assert dev < tol and drift < tol / 4, (dev, drift)


# --- precision-and-batching stress: 8192^2 shear wave and the uneven batch

@pytest.mark.parametrize("storage,rounding,tol", [("f32", "nearest", 1e-5), ("f16", "stochastic", 1e-4),
                                                  ("bf16", "stochastic", 1e-3)])
def test_shear_wave_8192_decays_as_closed_form(storage, rounding, tol):
    """u_x = u0 sin(2 pi y / N) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3;
    1000 steps on the full 8192^2 lattice, the profile averaged along x.

    The wave loses only 6e-5 of its amplitude in 1000 steps, 6e-10 per step,
    less than the spacing of the FP32 values that carry it (half an ulp of
    |d_i| ~ 3e-3 is 1.2e-10, ~7e-10 in u).  FP32 storage with FP32 arithmetic
    forms the small increment omega (feq - d) first and rounds d + increment
    once, so the decay is carried (measured 1.9e-7; relaxing the stored value
    directly lagged by 4.7e-5).  The 16-bit formats round stochastically:
    unbiased, and the errors average out along x (FP16 1.5e-5, BF16 7.7e-5)."""
    from paper_2006_12910_amd import inputs, lb
    n, tau, u0, steps = 8192, 0.8, 0.01, 1000
    gpu = lb.Domain(n, n, tau=tau, storage=storage, rounding=rounding,
                    init=inputs.shear_wave_field(n, n, u0, 1, 0.0))
    gpu.step(steps)
    _, ux, uy = gpu.moments()
    prof = ux.mean(axis=1)
    k = 2 * np.pi / n
    ref = u0 * np.sin(k * np.arange(n)) * np.exp(-(tau - 0.5) / 3 * k * k * steps)
    err = rel_l2(prof, ref)
    print(f"shear wave 8192^2 {storage}: profile vs closed form {err:.2e}, |uy| max {np.abs(uy).max():.1e}")
    assert err < tol, err


def test_stress_batch_members_equal_solo_runs():
    """The full 201-domain stress batch (FP16, stochastic rounding): sampled
    members, the largest included, evolve bit for bit as when run alone."""
    from paper_2006_12910_amd import inputs, lb
    specs = [dict(n=8192, tau=0.8, k=1, phase=0.0, obstacle_seed=None)] + inputs.stress_batch(count=200, seed=0)

    def dom(spec):
        n = spec["n"]
        mask = None if spec["obstacle_seed"] is None else inputs.stress_obstacles(n, spec["obstacle_seed"])
        return lb.Domain(n, n, tau=spec["tau"], storage="f16", rounding="stochastic", obstacles=mask,
                         init=inputs.shear_wave_field(n, n, 0.01, spec["k"], spec["phase"]))

    doms = [dom(s) for s in specs]
    batch = lb.Batch(doms)
    batch.step(20)
    order = sorted(range(1, 201), key=lambda i: specs[i]["n"])
    for i in [0, order[0], order[100], order[-1]]:
        solo = dom(specs[i])
        solo.step(20)
        assert np.array_equal(solo.populations(), doms[i].populations()), specs[i]["n"]
        solo.close()
    batch.close()
