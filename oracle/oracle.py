"""ctypes wrapper of the CPU oracle (oracle/liblbo.so).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy float64 in row-major [ny][nx]
order; populations are [9][ny][nx] with the paper's direction order
(Sec. 2: rest, +x, +y, -x, -y, then the diagonals (1,1), (-1,1), (-1,-1), (1,-1)).
"""
import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

PERIODIC, WALL, PRESSURE = 0, 1, 2
PARTICLE_FIXED = 1


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32),
        ("rho_in", C.c_double), ("rho_out", C.c_double),
        ("tau", C.c_double), ("rho0", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
        ("kT", C.c_double), ("seed", C.c_uint64), ("domain_id", C.c_uint32),
        ("power_law", C.c_int32), ("n_index", C.c_double), ("K", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double),
        ("lj_psi", C.c_double), ("lj_rit", C.c_double), ("lj_floor", C.c_double),
        ("force_average", C.c_int32), ("trt", C.c_int32), ("magic", C.c_double),
    ]


class _Particle(C.Structure):
    _fields_ = [
        ("x", C.c_double), ("y", C.c_double), ("radius", C.c_double),
        ("density_ratio", C.c_double), ("ux", C.c_double), ("uy", C.c_double),
        ("omega", C.c_double), ("fx", C.c_double), ("fy", C.c_double),
        ("torque", C.c_double), ("flags", C.c_int32), ("pad_", C.c_int32),
    ]


class _Params3(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("wall_x", C.c_int32), ("wall_y", C.c_int32), ("wall_z", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
        ("gz", C.c_double), ("trt", C.c_int32), ("magic", C.c_double), ("q", C.c_int32),
        ("power_law", C.c_int32), ("n_index", C.c_double), ("K", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double), ("kT", C.c_double),
        ("seed", C.c_uint64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or any(os.path.getmtime(path) < os.path.getmtime(src)
                                       for src in _build.SOURCES):
        _build.build()
    lib = C.CDLL(path)
    P = C.POINTER
    dptr = P(C.c_double)
    lib.lbo_create.restype = C.c_void_p
    lib.lbo_create.argtypes = [P(_Params), P(C.c_uint8), dptr, dptr, dptr]
    lib.lbo_destroy.argtypes = [C.c_void_p]
    lib.lbo_add_particle.restype = C.c_int
    lib.lbo_add_particle.argtypes = [C.c_void_p, P(_Particle)]
    lib.lbo_run.argtypes = [C.c_void_p, C.c_int64]
    lib.lbo_time.restype = C.c_int64
    lib.lbo_time.argtypes = [C.c_void_p]
    lib.lbo_moments.argtypes = [C.c_void_p, dptr, dptr, dptr]
    lib.lbo_populations.argtypes = [C.c_void_p, dptr]
    lib.lbo_set_populations.argtypes = [C.c_void_p, dptr]
    lib.lbo_labels.argtypes = [C.c_void_p, P(C.c_uint8)]
    lib.lbo_num_particles.restype = C.c_int
    lib.lbo_num_particles.argtypes = [C.c_void_p]
    lib.lbo_get_particles.argtypes = [C.c_void_p, P(_Particle)]
    lib.lbo_mass.restype = C.c_double
    lib.lbo_mass.argtypes = [C.c_void_p]
    lib.lbo_momentum.argtypes = [C.c_void_p, dptr, dptr]
    lib.lbo_link_forces.argtypes = [C.c_void_p, dptr]
    lib.lbo_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    lib.lbo_logf.restype = C.c_float
    lib.lbo_logf.argtypes = [C.c_float]
    lib.lbo_sincos2pi.argtypes = [C.c_float, P(C.c_float), P(C.c_float)]
    lib.lbo_normals_block.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                      P(C.c_float)]
    lib.lbo_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P(C.c_float)]
    lib.lbo_normals_bulk.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                     P(C.c_float)]
    lib.lbo3_create.restype = C.c_void_p
    lib.lbo3_create.argtypes = [P(_Params3), P(C.c_uint8), dptr, dptr, dptr, dptr]
    lib.lbo3_destroy.argtypes = [C.c_void_p]
    lib.lbo3_run.argtypes = [C.c_void_p, C.c_int64]
    lib.lbo3_time.restype = C.c_int64
    lib.lbo3_time.argtypes = [C.c_void_p]
    lib.lbo3_moments.argtypes = [C.c_void_p, dptr, dptr, dptr, dptr]
    lib.lbo3_populations.argtypes = [C.c_void_p, dptr]
    lib.lbo3_mass.restype = C.c_double
    lib.lbo3_mass.argtypes = [C.c_void_p]
    lib.lbo3_momentum.argtypes = [C.c_void_p, dptr]
    lib.lbo3_lattice.argtypes = [C.c_int, P(C.c_int), P(C.c_int), P(C.c_int), dptr]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


@dataclass
class OracleParams:
    nx: int
    ny: int
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    rho_in: float = 1.0
    rho_out: float = 1.0
    tau: float = 1.0
    rho0: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    kT: float = 0.0
    seed: int = 0
    domain_id: int = 0
    power_law: bool = False
    n_index: float = 1.0
    K: float = 0.0
    tau_min: float = 0.51
    tau_max: float = 2.5
    lj_psi: float = 20.0
    lj_rit: float = 2.5
    lj_floor: float = 0.1
    force_average: bool = False  # mean of this and the previous step's force in Eq. MP5
    trt: bool = False  # two relaxation times, (tau - 1/2)(tau_minus - 1/2) = magic (no noise)
    magic: float = 3.0 / 16.0
    extra: dict = field(default_factory=dict)


class Oracle:
    """One simulated domain of the FP64 CPU oracle."""

    def __init__(self, prm: OracleParams, obstacles=None, rho=None, ux=None, uy=None):
        lib = _load()
        self.prm = prm
        self.nx, self.ny = prm.nx, prm.ny
        c = _Params(prm.nx, prm.ny, prm.bc_x, prm.bc_y, prm.rho_in, prm.rho_out, prm.tau,
                    prm.rho0, prm.gx, prm.gy, prm.kT, prm.seed & (2**64 - 1),
                    prm.domain_id & 0xFFFFFFFF, int(prm.power_law), prm.n_index, prm.K,
                    prm.tau_min, prm.tau_max, prm.lj_psi, prm.lj_rit, prm.lj_floor,
                    int(prm.force_average), int(prm.trt), prm.magic)
        shape = (prm.ny, prm.nx)
        mask = None
        if obstacles is not None:
            self._mask = np.ascontiguousarray(obstacles, dtype=np.uint8).reshape(shape)
            mask = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        fields = []
        for a in (rho, ux, uy):
            fields.append(None if a is None else np.ascontiguousarray(a, np.float64).reshape(shape))
        self._h = lib.lbo_create(C.byref(c), mask, *[_dp(a) for a in fields])
        if not self._h:
            raise ValueError("oracle rejected parameters")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.lbo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_particle(self, x, y, radius, density_ratio=1.0, ux=0.0, uy=0.0, omega=0.0,
                     fixed=False):
        p = _Particle(x, y, radius, density_ratio, ux, uy, omega, 0, 0, 0,
                      PARTICLE_FIXED if fixed else 0, 0)
        if self._lib.lbo_add_particle(self._h, C.byref(p)) != 0:
            raise ValueError("particle overlaps a solid or another particle")

    def run(self, nsteps):
        self._lib.lbo_run(self._h, int(nsteps))
        return self

    @property
    def t(self):
        return self._lib.lbo_time(self._h)

    def moments(self):
        shape = (self.ny, self.nx)
        r, u, v = (np.zeros(shape) for _ in range(3))
        self._lib.lbo_moments(self._h, _dp(r), _dp(u), _dp(v))
        return r, u, v

    def populations(self):
        f = np.zeros((9, self.ny, self.nx))
        self._lib.lbo_populations(self._h, _dp(f))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(9, self.ny, self.nx)
        self._lib.lbo_set_populations(self._h, _dp(f))

    def labels(self):
        out = np.zeros((self.ny, self.nx), np.uint8)
        self._lib.lbo_labels(self._h, out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out

    def particles(self):
        n = self._lib.lbo_num_particles(self._h)
        arr = (_Particle * max(n, 1))()
        self._lib.lbo_get_particles(self._h, arr)
        keys = ["x", "y", "radius", "density_ratio", "ux", "uy", "omega", "fx", "fy", "torque"]
        return np.array([[getattr(arr[i], k) for k in keys] for i in range(n)]).reshape(n, 10)

    def link_forces(self):
        """[np][6]: exterior-side (Fx, Fy, T), then interior-side (Fx, Fy, T)."""
        n = self._lib.lbo_num_particles(self._h)
        out = np.zeros((max(n, 1), 6))
        self._lib.lbo_link_forces(self._h, _dp(out))
        return out[:n]

    def mass(self):
        return self._lib.lbo_mass(self._h)

    def momentum(self):
        a, b = C.c_double(), C.c_double()
        self._lib.lbo_momentum(self._h, C.byref(a), C.byref(b))
        return a.value, b.value


def philox4x32_10(ctr, key):
    lib = _load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib.lbo_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def normals(seed, domain_id, node, step):
    lib = _load()
    o = (C.c_float * 6)()
    lib.lbo_normals(seed & (2**64 - 1), domain_id & 0xFFFFFFFF, node & 0xFFFFFFFF,
                    step & 0xFFFFFFFF, o)
    return np.array([o[i] for i in range(6)], dtype=np.float32)


def normals_block(seed, domain_id, node, step, block):
    """The six FP32 normals of Philox block `block` of (node, step)."""
    o = (C.c_float * 6)()
    _load().lbo_normals_block(seed & (2**64 - 1), domain_id & 0xFFFFFFFF, node & 0xFFFFFFFF,
                              step & 0xFFFFFFFF, block & 0xFFFFFFFF, o)
    return np.array([o[i] for i in range(6)], dtype=np.float32)


def normals_bulk(seed, domain_id, step, node0, count):
    """[count][6] FP32 normals of nodes node0 .. node0+count-1 at `step`."""
    out = np.empty((count, 6), dtype=np.float32)
    _load().lbo_normals_bulk(seed & (2**64 - 1), domain_id & 0xFFFFFFFF, step & 0xFFFFFFFF,
                             node0 & 0xFFFFFFFF, count,
                             out.ctypes.data_as(C.POINTER(C.c_float)))
    return out


def own_logf(u):
    return np.float32(_load().lbo_logf(float(u)))


def own_sincos2pi(u):
    s, c = C.c_float(), C.c_float()
    _load().lbo_sincos2pi(float(u), C.byref(s), C.byref(c))
    return np.float32(s.value), np.float32(c.value)


class Oracle3:
    """One D3Q19 or D3Q27 domain of the FP64 CPU oracle (lbo3.c).  Node arrays
    are [nz][ny][nx]; populations [q][nz][ny][nx]."""

    def __init__(self, nx, ny, nz, tau=1.0, rho0=1.0, g=(0.0, 0.0, 0.0), walls=(False, False, False),
                 obstacles=None, init=None, collision="bgk", magic=3.0 / 16.0, lattice="d3q19",
                 power_law=None, kT=0.0, seed=0):
        """collision "trt": two relaxation times, (tau - 1/2)(tau_minus - 1/2) = magic;
        lattice "d3q19" or "d3q27"; power_law: dict(n, K, tau_min=0.51, tau_max=2.5);
        kT > 0: thermal noise (BGK only) keyed by seed."""
        lib = _load()
        self.nx, self.ny, self.nz = nx, ny, nz
        self.q = {"d3q19": 19, "d3q27": 27}[lattice]
        pl = power_law or {}
        c = _Params3(nx, ny, nz, int(walls[0]), int(walls[1]), int(walls[2]), tau, rho0, *g,
                     int(collision == "trt"), magic, self.q, int(power_law is not None),
                     pl.get("n", 1.0), pl.get("K", 0.0), pl.get("tau_min", 0.51),
                     pl.get("tau_max", 2.5), kT, seed)
        shape = (nz, ny, nx)
        mask = None
        if obstacles is not None:
            self._mask = np.ascontiguousarray(obstacles, dtype=np.uint8).reshape(shape)
            mask = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        fields = [None] * 4
        if init is not None:
            fields = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))
                      for a in init]
        self._h = lib.lbo3_create(C.byref(c), mask, *[_dp(a) for a in fields])
        if not self._h:
            raise ValueError("oracle rejected parameters")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.lbo3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, nsteps):
        self._lib.lbo3_run(self._h, int(nsteps))
        return self

    @property
    def t(self):
        return self._lib.lbo3_time(self._h)

    def moments(self):
        shape = (self.nz, self.ny, self.nx)
        out = [np.zeros(shape) for _ in range(4)]
        self._lib.lbo3_moments(self._h, *[_dp(a) for a in out])
        return tuple(out)

    def populations(self):
        f = np.zeros((self.q, self.nz, self.ny, self.nx))
        self._lib.lbo3_populations(self._h, _dp(f))
        return f

    def mass(self):
        return self._lib.lbo3_mass(self._h)

    def momentum(self):
        j = np.zeros(3)
        self._lib.lbo3_momentum(self._h, _dp(j))
        return j


def lattice3(q=19):
    """(ex, ey, ez, w) of the oracle's D3Q19 or D3Q27 velocity set."""
    lib = _load()
    ex, ey, ez = (C.c_int * q)(), (C.c_int * q)(), (C.c_int * q)()
    w = np.zeros(q)
    lib.lbo3_lattice(q, ex, ey, ez, _dp(w))
    return np.array(ex[:]), np.array(ey[:]), np.array(ez[:]), w
