"""Shared helpers of the parity tests: build the GPU domain and the oracle
from one parameter set, and compare their outputs."""
import numpy as np

from oracle import Oracle, OracleParams
from oracle.oracle import PERIODIC, PRESSURE, WALL

_BC = {"periodic": PERIODIC, "wall": WALL, "pressure": PRESSURE}


def make_pair(nx, ny, storage="f64", bc_x="periodic", bc_y="periodic", tau=1.0, g=(0.0, 0.0),
              rho0=1.0, rho_in=1.0, rho_out=1.0, kT=0.0, seed=0, domain_id=0, power_law=None,
              obstacles=None, particles=(), init=None, lj=(20.0, 2.5, 0.1), max_particles=None,
              rounding="nearest", compute="native", force_average=False, collision="bgk",
              magic=3.0 / 16.0):
    """(gpu Domain, Oracle) with identical parameters and inputs."""
    from paper_2006_12910_amd import lb
    plist = list(particles)
    nmax = len(plist) if max_particles is None else max_particles
    gpu = lb.Domain(nx, ny, tau=tau, rho0=rho0, g=g, bc_x=bc_x, bc_y=bc_y, storage=storage,
                    rounding=rounding, compute=compute, rho_in=rho_in, rho_out=rho_out, kT=kT, seed=seed,
                    domain_id=domain_id, power_law=power_law, obstacles=obstacles,
                    max_particles=nmax, lj=lj, init=init, collision=collision, magic=magic)
    if force_average:
        gpu.set_option(lb.OPT_FORCE_AVERAGE, 1)
    pl = power_law or {}
    prm = OracleParams(nx=nx, ny=ny, bc_x=_BC[bc_x], bc_y=_BC[bc_y], rho_in=rho_in,
                       rho_out=rho_out, tau=tau, rho0=rho0, gx=g[0], gy=g[1], kT=kT, seed=seed,
                       domain_id=domain_id, power_law=power_law is not None,
                       n_index=pl.get("n", 1.0), K=pl.get("K", 0.0),
                       tau_min=pl.get("tau_min", 0.51), tau_max=pl.get("tau_max", 2.5),
                       lj_psi=lj[0], lj_rit=lj[1], lj_floor=lj[2], force_average=force_average,
                       trt=collision == "trt", magic=magic)
    fields = (None, None, None) if init is None else tuple(
        np.broadcast_to(np.asarray(a, np.float64), (ny, nx)) for a in init)
    ora = Oracle(prm, obstacles, *fields)
    if plist:
        gpu.add_particles(plist)
        for p in plist:
            ora.add_particle(p["x"], p["y"], p["radius"], p.get("density_ratio", 1.0),
                             p.get("ux", 0.0), p.get("uy", 0.0), p.get("omega", 0.0),
                             fixed=p.get("fixed", False))
    return gpu, ora


def rel_l2(a, b):
    den = np.sqrt((np.asarray(b) ** 2).sum())
    return np.sqrt(((np.asarray(a) - np.asarray(b)) ** 2).sum()) / (den if den > 0 else 1.0)


def velocity_error(gpu, ora):
    """(max |rho_gpu - rho_oracle|, relative L2 of the velocity field)."""
    rg, ug, vg = gpu.moments()
    ro, uo, vo = ora.moments()
    num = np.sqrt(((ug - uo) ** 2 + (vg - vo) ** 2).sum())
    den = np.sqrt((uo ** 2 + vo ** 2).sum())
    return np.abs(rg - ro).max(), num / (den if den > 0 else 1.0)


def random_fields(nx, ny, seed, du=0.03, drho=0.01):
    rng = np.random.default_rng(seed)
    return (1.0 + drho * rng.standard_normal((ny, nx)), du * rng.standard_normal((ny, nx)),
            du * rng.standard_normal((ny, nx)))


def velocity_max_error(gpu, ora):
    """Element-wise velocity error relative to the oracle's largest speed:
    max_x |u_gpu - u_oracle| / max_x |u_oracle|.  A relative L2 over millions
    of nodes can hide an error confined to a few nodes (near a particle, say);
    this cannot."""
    _, ug, vg = gpu.moments()
    _, uo, vo = ora.moments()
    d = np.sqrt((ug - uo) ** 2 + (vg - vo) ** 2).max()
    s = np.sqrt(uo ** 2 + vo ** 2).max()
    return d / (s if s > 0 else 1.0)
