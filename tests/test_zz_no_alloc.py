"""lb_mass_static (the density sum for callers that cannot allocate: partial
sums in the library's fixed device array) against lb_mass, through the C ABI:
bit-identical on two calls in a row, the second on a smaller domain, and once
more on the first domain after the array held the second one's partials."""
import ctypes as C

import numpy as np
import pytest
import torch

from helpers import random_fields

pytestmark = pytest.mark.gpu


def _static_mass(lib, dom, out):
    rc = lib.lb_mass_static(dom.handle, C.c_void_p(out.data_ptr()))
    assert rc == 0, lib.lb_last_error().decode()
    torch.cuda.synchronize()
    return float(out.item())


def test_mass_static_equals_lb_mass_on_consecutive_calls():
    from paper_2006_12910_amd import lb
    lib = lb.library()
    big = lb.Domain(1030, 700, tau=0.9, storage="f32", init=random_fields(1030, 700, 3))
    small = lb.Domain(90, 41, tau=0.7, storage="f64", bc_y="wall",
                      init=random_fields(90, 41, 4))
    big.step(7)
    small.step(3)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    m_big = _static_mass(lib, big, out[0:1])
    assert m_big == big.mass()
    m_small = _static_mass(lib, small, out[1:2])  # smaller input, same array
    assert m_small == small.mass()
    assert _static_mass(lib, big, out[0:1]) == m_big
    assert np.isfinite(m_big) and abs(m_big / (1030 * 700) - 1) < 0.05
    # errors: null arguments, no work enqueued
    assert lib.lb_mass_static(big.handle, None) == lb.LB_EINVAL
    assert lib.lb_mass_static(None, C.c_void_p(out.data_ptr())) == lb.LB_EINVAL
    big.close()
    small.close()
