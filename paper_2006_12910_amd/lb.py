"""Python binding of liblb.so (include/lb.h): argument marshalling only.

Every computation runs in the HIP library; torch provides the device
workspace (a uint8 tensor the library sub-allocates) and the HIP stream.
Names follow the C ABI: ``Domain.step`` wraps ``lb_step``, ``Domain.moments``
wraps ``lb_moments`` and so on.
"""
import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime the library then shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblb.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_ESTATE, LB_EUNSTABLE, LB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PERIODIC, WALL, PRESSURE = 0, 1, 2
F64, F32, F16_DELTA, BF16_DELTA = 0, 1, 2, 3
ROUND_NEAREST, ROUND_STOCHASTIC = 0, 1
COMPUTE_NATIVE, COMPUTE_F64 = 0, 1
INIT_REST, INIT_FIELDS = 0, 1
BGK, TRT = 0, 1  # collisions of the 2D domains
LB3_BGK, LB3_TRT = 0, 1  # 3D collisions
LB3_D3Q19, LB3_D3Q27 = 0, 1
LB3_OPT_WIDE_OFFSETS = 1
PARTICLE_FIXED = 1
OPT_USE_GRAPH, OPT_TILE_WIDTH, OPT_ROWS_PER_THREAD, OPT_GRAPH_CHUNK, OPT_FORCE_AVERAGE = 1, 2, 3, 4, 5
OPT_TWO_STEP = 6
OPT_OVERLAP = 7
OPT_MASS_INTERVAL = 8
OPT_TWO_STEP_ROWS = 10
ABI_VERSION = 3

_BC = {"periodic": PERIODIC, "wall": WALL, "pressure": PRESSURE}
_ST = {"f64": F64, "f32": F32, "f16": F16_DELTA, "bf16": BF16_DELTA}
_RND = {"nearest": ROUND_NEAREST, "stochastic": ROUND_STOCHASTIC}

EXPORTED = [
    "lb_workspace_bytes", "lb_create_domain", "lb_set_obstacles", "lb_add_particles", "lb_step",
    "lb_moments", "lb_moments_device", "lb_moments_async", "lb_moments_wait", "lb_get_particles",
    "lb_mass", "lb_mass_static", "lb_set_mass_check", "lb_time",
    "lb_get_populations", "lb_set_populations", "lb_set_time", "lb_get_particle_state",
    "lb_set_particle_state", "lb_set_option", "lb_get_option",
    "lb_destroy_domain", "lb_batch_workspace_bytes", "lb_batch_create", "lb_batch_step",
    "lb_batch_set_option", "lb_batch_destroy", "lb_noise_normals", "lb_autotune",
    "lb_batch_autotune", "lb_batch_get_option",
    "lb3_workspace_bytes", "lb3_create_domain", "lb3_set_obstacles", "lb3_step", "lb3_moments",
    "lb3_get_populations", "lb3_mass", "lb3_time", "lb3_set_option", "lb3_destroy_domain",
    "lb_status_string", "lb_last_error",
]


class DomainDesc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("storage", C.c_int32),
        ("rounding", C.c_int32), ("compute", C.c_int32), ("obstacles", C.c_int32),
        ("max_particles", C.c_int32),
        ("power_law", C.c_int32), ("init_kind", C.c_int32), ("domain_id", C.c_uint32),
        ("seed", C.c_uint64), ("rho0", C.c_double), ("tau", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("rho_in", C.c_double), ("rho_out", C.c_double),
        ("kT", C.c_double), ("n_index", C.c_double), ("K", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double), ("lj_psi", C.c_double),
        ("lj_rit", C.c_double), ("lj_floor", C.c_double),
        ("init_rho", C.POINTER(C.c_double)), ("init_ux", C.POINTER(C.c_double)),
        ("init_uy", C.POINTER(C.c_double)),
        ("collision", C.c_int32), ("magic", C.c_double),
    ]


class Domain3Desc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("wall_x", C.c_int32), ("wall_y", C.c_int32), ("wall_z", C.c_int32),
        ("storage", C.c_int32), ("obstacles", C.c_int32), ("init_kind", C.c_int32),
        ("rho0", C.c_double), ("tau", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
        ("init_rho", C.POINTER(C.c_double)), ("init_ux", C.POINTER(C.c_double)),
        ("init_uy", C.POINTER(C.c_double)), ("init_uz", C.POINTER(C.c_double)),
        ("collision", C.c_int32), ("magic", C.c_double),
        ("rounding", C.c_int32), ("seed", C.c_uint64), ("lattice", C.c_int32),
        ("power_law", C.c_int32), ("n_index", C.c_double), ("K", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double), ("kT", C.c_double),
    ]


class Particle(C.Structure):
    _fields_ = [
        ("x", C.c_double), ("y", C.c_double), ("radius", C.c_double),
        ("density_ratio", C.c_double), ("ux", C.c_double), ("uy", C.c_double),
        ("omega", C.c_double), ("fx", C.c_double), ("fy", C.c_double), ("torque", C.c_double),
        ("flags", C.c_int32), ("reserved", C.c_int32),
    ]


class ParticleState(C.Structure):
    _fields_ = [("p", Particle), ("cover_fx", C.c_double), ("cover_fy", C.c_double),
                ("cover_torque", C.c_double)]


class LBError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def library():
    """Load liblb.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2006_12910_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, vp, st = C.POINTER, C.c_void_p, C.c_int32
    dp = P(C.c_double)
    sig = {
        "lb_workspace_bytes": [P(DomainDesc), P(C.c_size_t)],
        "lb_create_domain": [P(DomainDesc), vp, C.c_size_t, vp, P(vp)],
        "lb_set_obstacles": [vp, P(C.c_uint8), C.c_size_t],
        "lb_add_particles": [vp, P(Particle), st, P(st)],
        "lb_step": [vp, C.c_int64],
        "lb_moments": [vp, dp, dp, dp],
        "lb_moments_device": [vp, vp, vp, vp],
        "lb_moments_async": [vp, vp, vp, vp, vp, vp],
        "lb_moments_wait": [vp],
        "lb_get_particles": [vp, P(Particle), st],
        "lb_mass": [vp, dp],
        "lb_set_mass_check": [vp, C.c_double],
        "lb_mass_static": [vp, vp],
        "lb_time": [vp, P(C.c_int64)],
        "lb_get_populations": [vp, dp],
        "lb_set_populations": [vp, dp],
        "lb_set_time": [vp, C.c_int64],
        "lb_get_particle_state": [vp, P(ParticleState), st],
        "lb_set_particle_state": [vp, P(ParticleState), st],
        "lb_set_option": [vp, st, C.c_int64],
        "lb_get_option": [vp, st, P(C.c_int64)],
        "lb_destroy_domain": [vp],
        "lb_batch_workspace_bytes": [P(vp), st, P(C.c_size_t)],
        "lb_batch_create": [P(vp), st, vp, C.c_size_t, vp, P(vp)],
        "lb_batch_step": [vp, C.c_int64],
        "lb_batch_set_option": [vp, st, C.c_int64],
        "lb_batch_destroy": [vp],
        "lb_noise_normals": [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, st, vp,
                             vp],
        "lb_autotune": [vp, st, dp],
        "lb_batch_autotune": [vp, st, dp],
        "lb_batch_get_option": [vp, st, P(C.c_int64)],
        "lb3_workspace_bytes": [P(Domain3Desc), P(C.c_size_t)],
        "lb3_create_domain": [P(Domain3Desc), vp, C.c_size_t, vp, P(vp)],
        "lb3_set_obstacles": [vp, P(C.c_uint8), C.c_size_t],
        "lb3_step": [vp, C.c_int64],
        "lb3_moments": [vp, dp, dp, dp, dp],
        "lb3_get_populations": [vp, dp],
        "lb3_mass": [vp, dp],
        "lb3_time": [vp, P(C.c_int64)],
        "lb3_set_option": [vp, C.c_int32, C.c_int64],
        "lb3_destroy_domain": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = st
    lib.lb_status_string.restype = C.c_char_p
    lib.lb_status_string.argtypes = [st]
    lib.lb_last_error.restype = C.c_char_p
    lib.lb_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status, where):
    if status != LB_OK:
        lib = library()
        raise LBError(status, where, lib.lb_last_error().decode() or
                      lib.lb_status_string(status).decode())


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Domain:
    """One lattice domain on the GPU (lb_create_domain ... lb_destroy_domain)."""

    def __init__(self, nx, ny, *, tau=1.0, rho0=1.0, g=(0.0, 0.0), bc_x="periodic",
                 bc_y="periodic", storage="f32", rounding="nearest", compute="native",
                 rho_in=1.0, rho_out=1.0,
                 kT=0.0, seed=0, domain_id=0, power_law=None, obstacles=None, max_particles=0,
                 lj=(20.0, 2.5, 0.1), init=None, collision="bgk", magic=3.0 / 16.0, device="cuda",
                 stream=None):
        """collision "trt": two relaxation times, (tau - 1/2)(tau_minus - 1/2) = magic."""
        lib = library()
        d = DomainDesc()
        d.collision = {"bgk": BGK, "trt": TRT}[collision]
        d.magic = float(magic)
        d.abi_version = ABI_VERSION
        d.nx, d.ny = int(nx), int(ny)
        d.bc_x, d.bc_y = _BC[bc_x], _BC[bc_y]
        d.storage = _ST[storage]
        d.rounding = _RND[rounding]
        d.compute = {"native": COMPUTE_NATIVE, "f64": COMPUTE_F64}[compute]
        d.obstacles = 1 if obstacles is not None else 0
        d.max_particles = int(max_particles)
        d.domain_id = int(domain_id) & 0xFFFFFFFF
        d.seed = int(seed) & (2 ** 64 - 1)
        d.rho0, d.tau = float(rho0), float(tau)
        d.gx, d.gy = float(g[0]), float(g[1])
        d.rho_in, d.rho_out = float(rho_in), float(rho_out)
        d.kT = float(kT)
        if power_law is not None:
            d.power_law = 1
            d.n_index = float(power_law["n"])
            d.K = float(power_law["K"])
            d.tau_min = float(power_law.get("tau_min", 0.51))
            d.tau_max = float(power_law.get("tau_max", 2.5))
        d.lj_psi, d.lj_rit, d.lj_floor = (float(v) for v in lj)
        self._fields = None
        if init is not None:
            shape = (ny, nx)
            self._fields = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))
                            for a in init]
            d.init_kind = INIT_FIELDS
            d.init_rho, d.init_ux, d.init_uy = (_dptr(a) for a in self._fields)
        self.desc = d
        self.nx, self.ny = int(nx), int(ny)
        self._np = 0
        self._report_refs = []  # buffers of an asynchronous moment copy in flight
        nbytes = C.c_size_t()
        _check(lib.lb_workspace_bytes(C.byref(d), C.byref(nbytes)), "lb_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        self._stream = stream
        h = C.c_void_p()
        _check(lib.lb_create_domain(C.byref(d), C.c_void_p(self.workspace.data_ptr()),
                                    nbytes.value, _stream_ptr(stream), C.byref(h)),
               "lb_create_domain")
        self._h = h
        self._fields = None
        d.init_rho = d.init_ux = d.init_uy = None
        if obstacles is not None:
            self.set_obstacles(obstacles)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _check(library().lb_destroy_domain(self._h), "lb_destroy_domain")
            self._h = None
            self._report_refs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_obstacles(self, mask):
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8).reshape(self.ny, self.nx)
        _check(library().lb_set_obstacles(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                          m.size), "lb_set_obstacles")

    def add_particles(self, particles):
        """particles: iterable of dicts with x, y, radius and optional
        density_ratio, ux, uy, omega, fixed."""
        plist = list(particles)
        arr = (Particle * max(len(plist), 1))()
        for k, p in enumerate(plist):
            arr[k] = Particle(p["x"], p["y"], p["radius"], p.get("density_ratio", 1.0),
                              p.get("ux", 0.0), p.get("uy", 0.0), p.get("omega", 0.0), 0, 0, 0,
                              PARTICLE_FIXED if p.get("fixed") else 0, 0)
        first = C.c_int32()
        _check(library().lb_add_particles(self._h, arr, len(plist), C.byref(first)),
               "lb_add_particles")
        self._np = first.value + len(plist)
        return first.value

    def step(self, n=1):
        _check(library().lb_step(self._h, int(n)), "lb_step")
        return self

    def moments(self):
        shape = (self.ny, self.nx)
        r, u, v = (np.empty(shape) for _ in range(3))
        _check(library().lb_moments(self._h, _dptr(r), _dptr(u), _dptr(v)), "lb_moments")
        return r, u, v

    def moments_device(self):
        t = torch.empty((3, self.ny, self.nx), dtype=torch.float64, device=self.workspace.device)
        _check(library().lb_moments_device(self._h, C.c_void_p(t[0].data_ptr()),
                                           C.c_void_p(t[1].data_ptr()),
                                           C.c_void_p(t[2].data_ptr())), "lb_moments_device")
        return t

    def moments_async(self, stage, rho, ux, uy, copy_stream):
        """Moments of the current state into ``stage`` (device float64, at least
        3 ny nx elements) on the domain's stream, copied on ``copy_stream`` (a
        torch.cuda.Stream other than the domain's) into the pinned host float64
        tensors ``rho``, ``ux``, ``uy`` of shape (ny, nx).  Returns at once;
        ``moments_wait()`` blocks until the copy has landed.  The tensors are
        held until then."""
        n = self.ny * self.nx
        if not (stage.is_cuda and stage.dtype == torch.float64 and stage.is_contiguous()
                and stage.numel() >= 3 * n):
            raise ValueError("stage: contiguous device float64 tensor of >= 3 ny nx elements")
        for h in (rho, ux, uy):
            if (h.is_cuda or h.dtype != torch.float64 or tuple(h.shape) != (self.ny, self.nx)
                    or not h.is_contiguous() or not h.is_pinned()):
                raise ValueError("host arrays: pinned contiguous float64 tensors of shape (ny, nx)")
        _check(library().lb_moments_async(
            self._h, C.c_void_p(stage.data_ptr()), C.c_void_p(rho.data_ptr()),
            C.c_void_p(ux.data_ptr()), C.c_void_p(uy.data_ptr()),
            C.c_void_p(copy_stream.cuda_stream)), "lb_moments_async")
        self._report_refs.append((stage, rho, ux, uy, copy_stream))

    def moments_wait(self):
        _check(library().lb_moments_wait(self._h), "lb_moments_wait")
        self._report_refs = []

    def particles(self, n=None):
        """[n][10]: x, y, radius, density_ratio, ux, uy, omega, fx, fy, torque."""
        n = self.num_particles if n is None else n
        arr = (Particle * max(n, 1))()
        _check(library().lb_get_particles(self._h, arr, n), "lb_get_particles")
        keys = ["x", "y", "radius", "density_ratio", "ux", "uy", "omega", "fx", "fy", "torque"]
        return np.array([[getattr(arr[i], k) for k in keys] for i in range(n)]).reshape(n, 10)

    @property
    def num_particles(self):
        return self._np

    def mass(self):
        m = C.c_double()
        _check(library().lb_mass(self._h, C.byref(m)), "lb_mass")
        return m.value

    def set_mass_check(self, rel_tol):
        """Latch LB_EUNSTABLE when a call's final density sum drifts from the
        current one by more than rel_tol (relative); 0 switches it off."""
        _check(library().lb_set_mass_check(self._h, float(rel_tol)), "lb_set_mass_check")

    @property
    def time(self):
        t = C.c_int64()
        _check(library().lb_time(self._h, C.byref(t)), "lb_time")
        return t.value

    def populations(self):
        """Post-collision deviations f*_i - w_i rho0, [9][ny][nx] FP64."""
        f = np.empty((9, self.ny, self.nx))
        _check(library().lb_get_populations(self._h, _dptr(f)), "lb_get_populations")
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(9, self.ny, self.nx)
        _check(library().lb_set_populations(self._h, _dptr(f)), "lb_set_populations")

    def set_time(self, t):
        _check(library().lb_set_time(self._h, int(t)), "lb_set_time")

    def particle_state(self):
        """Checkpoint record of every particle (a ctypes array of
        ParticleState, for set_particle_state)."""
        n = self.num_particles
        arr = (ParticleState * max(n, 1))()
        _check(library().lb_get_particle_state(self._h, arr, n), "lb_get_particle_state")
        return arr, n

    def set_particle_state(self, state):
        arr, n = state
        _check(library().lb_set_particle_state(self._h, arr, int(n)), "lb_set_particle_state")
        self._np = int(n)

    def set_option(self, key, value):
        _check(library().lb_set_option(self._h, int(key), int(value)), "lb_set_option")

    def get_option(self, key):
        v = C.c_int64()
        _check(library().lb_get_option(self._h, int(key), C.byref(v)), "lb_get_option")
        return v.value

    def autotune(self, steps=20):
        ms = C.c_double()
        _check(library().lb_autotune(self._h, int(steps), C.byref(ms)), "lb_autotune")
        return ms.value


class Batch:
    """Several domains advanced together (lb_batch_create ... lb_batch_destroy)."""

    def __init__(self, domains, stream=None):
        lib = library()
        self.domains = list(domains)
        hs = (C.c_void_p * len(self.domains))(*[d.handle.value for d in self.domains])
        nbytes = C.c_size_t()
        _check(lib.lb_batch_workspace_bytes(hs, len(self.domains), C.byref(nbytes)),
               "lb_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8,
                                     device=self.domains[0].workspace.device)
        h = C.c_void_p()
        _check(lib.lb_batch_create(hs, len(self.domains), C.c_void_p(self.workspace.data_ptr()),
                                   nbytes.value, _stream_ptr(stream), C.byref(h)),
               "lb_batch_create")
        self._h = h

    def step(self, n=1):
        _check(library().lb_batch_step(self._h, int(n)), "lb_batch_step")
        return self

    def set_option(self, key, value):
        _check(library().lb_batch_set_option(self._h, int(key), int(value)), "lb_batch_set_option")

    def get_option(self, key):
        v = C.c_int64()
        _check(library().lb_batch_get_option(self._h, int(key), C.byref(v)), "lb_batch_get_option")
        return v.value

    def autotune(self, steps=8):
        """lb_batch_autotune: the two-step tile height (0.0 when cached or
        not applicable, else the best ms per step)."""
        ms = C.c_double()
        _check(library().lb_batch_autotune(self._h, int(steps), C.byref(ms)), "lb_batch_autotune")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            _check(library().lb_batch_destroy(self._h), "lb_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def noise_normals(seed, domain_id, step, node0, count, fp32_arithmetic=False, device="cuda"):
    """lb_noise_normals: Theta_3..Theta_8 of nodes node0.. at `step`, [count][6]
    FP32; fp32_arithmetic selects the transform of FP32-arithmetic collisions."""
    out = torch.empty((count, 6), dtype=torch.float32, device=device)
    _check(library().lb_noise_normals(int(seed) & (2 ** 64 - 1), int(domain_id) & 0xFFFFFFFF,
                                      int(step) & 0xFFFFFFFF, int(node0) & 0xFFFFFFFF,
                                      int(count), int(bool(fp32_arithmetic)),
                                      C.c_void_p(out.data_ptr()),
                                      _stream_ptr(None)), "lb_noise_normals")
    return out


class Domain3:
    """One D3Q19 or D3Q27 domain on the GPU (lb3_create_domain ...
    lb3_destroy_domain).  Node arrays are [nz][ny][nx]; populations
    [q][nz][ny][nx]."""

    def __init__(self, nx, ny, nz, *, tau=1.0, rho0=1.0, g=(0.0, 0.0, 0.0),
                 walls=(False, False, False), storage="f32", obstacles=None, init=None,
                 collision="bgk", magic=3.0 / 16.0, rounding=None, seed=0, lattice="d3q19",
                 power_law=None, kT=0.0, device="cuda", stream=None):
        """collision "trt": two relaxation times, (tau - 1/2)(tau_minus - 1/2) = magic.
        storage "f64" | "f32" | "f16" | "bf16"; rounding "nearest" | "stochastic"
        (16-bit storage only; its default there); lattice "d3q19" | "d3q27";
        power_law: dict(n, K, tau_min=0.51, tau_max=2.5); kT > 0: thermal noise
        (BGK or TRT), keyed by seed."""
        lib = library()
        d = Domain3Desc()
        d.abi_version = ABI_VERSION
        d.collision = {"bgk": LB3_BGK, "trt": LB3_TRT}[collision]
        d.lattice = {"d3q19": LB3_D3Q19, "d3q27": LB3_D3Q27}[lattice]
        if power_law is not None:
            d.power_law = 1
            d.n_index = float(power_law["n"])
            d.K = float(power_law["K"])
            d.tau_min = float(power_law.get("tau_min", 0.51))
            d.tau_max = float(power_law.get("tau_max", 2.5))
        self.q = 27 if lattice == "d3q27" else 19
        d.magic = float(magic)
        d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
        d.wall_x, d.wall_y, d.wall_z = (int(bool(w)) for w in walls)
        d.storage = _ST[storage]
        if rounding is None:
            rounding = "stochastic" if storage in ("f16", "bf16") else "nearest"
        d.rounding = _RND[rounding]
        d.seed = int(seed) & (2**64 - 1)
        d.kT = float(kT)
        d.obstacles = 1 if obstacles is not None else 0
        d.rho0, d.tau = float(rho0), float(tau)
        d.gx, d.gy, d.gz = (float(v) for v in g)
        shape = (nz, ny, nx)
        fields = None
        if init is not None:
            fields = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))
                      for a in init]
            d.init_kind = INIT_FIELDS
            d.init_rho, d.init_ux, d.init_uy, d.init_uz = (_dptr(a) for a in fields)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        nbytes = C.c_size_t()
        _check(lib.lb3_workspace_bytes(C.byref(d), C.byref(nbytes)), "lb3_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(lib.lb3_create_domain(C.byref(d), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                     _stream_ptr(stream), C.byref(h)), "lb3_create_domain")
        self._h = h
        del fields
        if obstacles is not None:
            m = np.ascontiguousarray(np.asarray(obstacles) != 0, dtype=np.uint8).reshape(shape)
            _check(lib.lb3_set_obstacles(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)), m.size),
                   "lb3_set_obstacles")

    def close(self):
        if getattr(self, "_h", None):
            _check(library().lb3_destroy_domain(self._h), "lb3_destroy_domain")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(library().lb3_step(self._h, int(n)), "lb3_step")
        return self

    def moments(self):
        shape = (self.nz, self.ny, self.nx)
        out = [np.empty(shape) for _ in range(4)]
        _check(library().lb3_moments(self._h, *[_dptr(a) for a in out]), "lb3_moments")
        return tuple(out)

    def populations(self):
        f = np.empty((self.q, self.nz, self.ny, self.nx))
        _check(library().lb3_get_populations(self._h, _dptr(f)), "lb3_get_populations")
        return f

    def mass(self):
        m = C.c_double()
        _check(library().lb3_mass(self._h, C.byref(m)), "lb3_mass")
        return m.value

    @property
    def time(self):
        t = C.c_int64()
        _check(library().lb3_time(self._h, C.byref(t)), "lb3_time")
        return t.value

    def set_option(self, option, value):
        _check(library().lb3_set_option(self._h, int(option), int(value)), "lb3_set_option")
        return self
