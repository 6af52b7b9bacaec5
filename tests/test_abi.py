"""The C-ABI library loads and exports every entry point include/lb.h
declares; argument validation needs no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    return sorted(set(re.findall(r"^(?:lb_status|const char \*)\s*(lb3?_\w+)\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for required in ("lb_create_domain", "lb_set_obstacles", "lb_add_particles", "lb_step",
                     "lb_moments", "lb_destroy_domain", "lb_batch_create", "lb_batch_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    names = declared_entry_points()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lb.EXPORTED)


def _desc(**kw):
    from paper_2006_12910_amd import lb
    d = lb.DomainDesc()
    d.abi_version, d.nx, d.ny, d.tau, d.rho0 = lb.ABI_VERSION, 64, 32, 0.8, 1.0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad,msg", [
    (dict(tau=0.5), "tau"), (dict(nx=2), "nx"), (dict(abi_version=1), "abi"),
    (dict(bc_y=2), "bc_y"), (dict(storage=9), "storage"), (dict(rounding=1), "stochastic"),
    (dict(max_particles=251), "max_particles"), (dict(kT=-1.0), "kT"),
    (dict(power_law=1, n_index=0.5, K=0.01, tau_min=0.4, tau_max=2.5), "power law"),
    (dict(bc_x=2, rho_in=0.0, rho_out=1.0), "pressure"), (dict(init_kind=1), "INIT_FIELDS"),
    (dict(compute=2), "compute"),
    # a population buffer must span fewer than 2^32 bytes (32-bit sweep offsets)
    (dict(nx=16384, ny=8192, storage=1), "too large"), (dict(nx=8192, ny=8192, storage=0), "too large"),
])
def test_validation_errors(bad, msg):
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    st = lib.lb_workspace_bytes(C.byref(_desc(**bad)), C.byref(n))
    assert st == lb.LB_EINVAL
    assert msg.lower() in lib.lb_last_error().decode().lower()


def test_binding_abi_version_matches_the_header():
    from paper_2006_12910_amd import lb
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    assert int(re.search(r"^#define LB_ABI_VERSION (\d+)u", src, re.M).group(1)) == lb.ABI_VERSION


def test_trt_validation():
    """The 2D collision option: an unknown collision or a non-positive magic
    number is LB_EINVAL; TRT with thermal noise is LB_EUNSUPPORTED."""
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    for kw, status, msg in ((dict(collision=2), lb.LB_EINVAL, "collision"),
                            (dict(collision=1, magic=0.0), lb.LB_EINVAL, "magic"),
                            (dict(collision=1, magic=0.25, kT=1e-5), lb.LB_EUNSUPPORTED, "noise")):
        assert lib.lb_workspace_bytes(C.byref(_desc(**kw)), C.byref(n)) == status
        assert msg in lib.lb_last_error().decode().lower()
    assert lib.lb_workspace_bytes(C.byref(_desc(collision=1, magic=0.25)), C.byref(n)) == 0


def test_largest_buffers_within_the_offset_limit_are_accepted():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    for nx, ny, storage in ((8192, 8192, 2), (8192, 8192, 1), (10880, 10880, 1), (15360, 15360, 3)):
        assert lib.lb_workspace_bytes(C.byref(_desc(nx=nx, ny=ny, storage=storage)), C.byref(n)) == 0
        assert n.value > 2 * 9 * nx * ny * (4 if storage == 1 else 2)


def test_workspace_size_covers_both_population_buffers():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    for storage, size in ((0, 8), (1, 4), (2, 2), (3, 2)):
        n = C.c_size_t()
        assert lib.lb_workspace_bytes(C.byref(_desc(storage=storage, nx=1000, ny=100)),
                                      C.byref(n)) == 0
        assert n.value >= 2 * 9 * 1024 * 100 * size


def test_null_arguments_are_rejected():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    assert lib.lb_step(None, 1) == lb.LB_EINVAL
    assert lib.lb_moments(None, None, None, None) == lb.LB_EINVAL
    assert lib.lb_moments_async(None, None, None, None, None, None) == lb.LB_EINVAL
    assert lib.lb_moments_wait(None) == lb.LB_EINVAL
    assert lib.lb_destroy_domain(None) == lb.LB_EINVAL
    assert lib.lb_status_string(lb.LB_EUNSTABLE).decode().startswith("simulation")


def test_binding_constants_match_the_header():
    """Every LB_* integer constant of include/lb.h has the same value in the
    Python binding (options, storage formats, boundaries, status codes)."""
    from paper_2006_12910_amd import lb
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"^#define (LB_OPT_\w+) (\d+)", src, re.M))
    assert "LB_OPT_TWO_STEP" in consts
    for name, value in consts.items():
        assert getattr(lb, name[len("LB_"):]) == value, name


def _desc3(**kw):
    from paper_2006_12910_amd import lb
    d = lb.Domain3Desc()
    d.abi_version, d.nx, d.ny, d.nz, d.tau, d.rho0, d.storage = lb.ABI_VERSION, 32, 16, 8, 0.8, 1.0, 1
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad,msg", [
    (dict(tau=0.5), "tau"), (dict(nz=2), "nz"), (dict(abi_version=1), "abi"),
    (dict(storage=4), "storage"), (dict(init_kind=1), "INIT_FIELDS"), (dict(rho0=0.0), "rho0"),
    (dict(rounding=2), "rounding"), (dict(rounding=1), "stochastic rounding needs"),
    (dict(lattice=2), "lattice"),
    (dict(collision=2), "collision"), (dict(collision=1, magic=0.0), "magic"),
    (dict(kT=-1e-5), "kT"), (dict(kT=float("nan")), "kT"), (dict(kT=float("inf")), "kT"),
])
def test_d3q19_validation_errors(bad, msg):
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    assert lib.lb3_workspace_bytes(C.byref(_desc3(**bad)), C.byref(n)) == lb.LB_EINVAL
    assert msg.lower() in lib.lb_last_error().decode().lower()


def test_d3q19_noise_needs_fewer_than_2_32_nodes():
    """Thermal noise on the 3D lattices (BGK or TRT): fewer than 2^32 nodes
    (the node number is the generator's 32-bit counter word)."""
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    assert lib.lb3_workspace_bytes(C.byref(_desc3(kT=1e-5, nx=2048, ny=2048, nz=1024)),
                                   C.byref(n)) == lb.LB_EUNSUPPORTED
    assert "2^32" in lib.lb_last_error().decode()
    for ok in (_desc3(kT=1e-5, nx=2048, ny=2048, nz=1023), _desc3(kT=1e-5, collision=1, magic=0.25)):
        assert lib.lb3_workspace_bytes(C.byref(ok), C.byref(n)) == 0


def test_d3q19_workspace_covers_both_population_buffers():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    for storage, size in ((0, 8), (1, 4), (2, 2), (3, 2)):
        for lattice, q in ((0, 19), (1, 27)):
            n = C.c_size_t()
            desc = _desc3(storage=storage, nx=100, ny=30, nz=20, lattice=lattice)
            assert lib.lb3_workspace_bytes(C.byref(desc), C.byref(n)) == 0
            assert n.value >= 2 * q * 128 * 30 * 20 * size
    assert lib.lb3_step(None, 1) == lb.LB_EINVAL
    assert lib.lb3_set_option(None, lb.LB3_OPT_WIDE_OFFSETS, 1) == lb.LB_EINVAL
    assert lib.lb3_destroy_domain(None) == lb.LB_EINVAL


def test_d3q19_lattices_beyond_32_bit_offsets_are_sized():
    """A lattice whose population buffer passes 2^32 bytes is admitted (the
    sweep then takes 64-bit offsets): the workspace holds both buffers."""
    from paper_2006_12910_amd import lb
    lib = lb.library()
    n = C.c_size_t()
    assert lib.lb3_workspace_bytes(C.byref(_desc3(nx=1024, ny=1024, nz=128)), C.byref(n)) == 0
    assert n.value >= 2 * 19 * 1024 * 1024 * 128 * 4 > 2 * 2 ** 32


def test_d3q19_option_constant_matches_the_header():
    from paper_2006_12910_amd import lb
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    assert int(re.search(r"^#define LB3_OPT_WIDE_OFFSETS (\d+)", src, re.M).group(1)) == \
        lb.LB3_OPT_WIDE_OFFSETS
