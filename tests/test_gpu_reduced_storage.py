"""Accuracy of FP16/BF16 deviation storage (FP32 arithmetic) against the FP64
oracle: relative L2 of the velocity after 1000 steps of a decaying shear wave
(u0 = 0.01) on a periodic domain.  Bounds: FP16 with stochastic rounding meets
the 1e-3 reduced-storage target; the other formats are held to the measured
error with margin (round-to-nearest 16-bit storage stagnates: updates smaller
than half an ulp are lost)."""
import json
import os

import numpy as np
import pytest

from helpers import make_pair, velocity_error

pytestmark = pytest.mark.gpu

BOUNDS = {("f16", "stochastic"): 1e-3, ("f16", "nearest"): 5e-2,
          ("bf16", "stochastic"): 1e-2, ("bf16", "nearest"): 5e-1, ("f32", "nearest"): 1e-5,
          ("f32", "stochastic"): 1e-5}


@pytest.mark.parametrize("tau", [0.55, 1.2])
@pytest.mark.parametrize("storage,rounding", list(BOUNDS))
def test_shear_wave_storage_error(storage, rounding, tau):
    n = 128
    y = np.arange(n)
    ux = np.tile((0.01 * np.sin(2 * np.pi * 2 * y / n + 0.3))[:, None], (1, n))
    gpu, ora = make_pair(n, n, storage=storage, rounding=rounding, tau=tau,
                         init=(np.ones((n, n)), ux, np.zeros((n, n))))
    gpu.step(1000)
    ora.run(1000)
    _, err = velocity_error(gpu, ora)
    print(f"{storage}/{rounding} tau {tau}: rel L2 {err:.3e}", flush=True)
    table = os.environ.get("LB_STORAGE_ERROR_TABLE")  # optional JSON-lines record of the errors
    if table:
        with open(table, "a") as fh:
            fh.write(json.dumps(dict(storage=storage, rounding=rounding, tau=tau, rel_l2=err)) + "\n")
    assert err < BOUNDS[(storage, rounding)], err
