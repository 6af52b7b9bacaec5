"""Pins of the oracle's thermal-noise generator (Sec. 4: six normal deviates
Theta_k per node and step; the generator itself is not given in the paper, so
a counter-based Philox4x32-10 with Box-Muller is used, each pinned below)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import normals, own_logf, own_sincos2pi, philox4x32_10

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert philox4x32_10(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 3


def test_own_log_accuracy():
    rng = np.random.default_rng(1)
    ks = np.concatenate([np.arange(0, 64), (1 << 21) - 1 - np.arange(64),
                         rng.integers(0, 1 << 21, 20000)])
    for k in ks:
        u = np.float32((2 * int(k) + 1) / 4194304.0)
        ref = np.log(np.float64(u))
        got = np.float64(own_logf(u))
        ulp = np.spacing(np.float32(abs(ref)))
        assert abs(got - ref) <= 3 * ulp, (k, got, ref)


def test_own_sincos_accuracy():
    rng = np.random.default_rng(2)
    ks = np.concatenate([np.arange(0, 32), (1 << 21) - 1 - np.arange(32),
                         np.array([1 << 19, (1 << 20), 3 << 19]) - 1,
                         rng.integers(0, 1 << 21, 20000)])
    for k in ks:
        u = np.float32((2 * int(k) + 1) / 4194304.0)
        s, c = own_sincos2pi(u)
        a = 2 * np.pi * np.float64(u)
        assert abs(np.float64(s) - np.sin(a)) < 3e-7
        assert abs(np.float64(c) - np.cos(a)) < 3e-7


def test_normals_statistics():
    z = np.array([normals(20061291, 7, node, step) for node in range(2500) for step in range(4)],
                 dtype=np.float64)
    assert z.shape == (10000, 6)
    flat = z.ravel()
    assert abs(flat.mean()) < 0.015
    assert abs(flat.var() - 1) < 0.02
    assert abs(stats.kurtosis(flat, fisher=False) - 3) < 0.1
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    for k in range(6):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-4
    corr = np.corrcoef(z.T)
    assert np.abs(corr - np.eye(6)).max() < 0.04


def test_normals_keying():
    a = normals(5, 0, 10, 3)
    assert np.array_equal(a, normals(5, 0, 10, 3))
    for other in (normals(5, 0, 11, 3), normals(5, 0, 10, 4), normals(5, 1, 10, 3),
                  normals(6, 0, 10, 3), normals(5 + (1 << 32), 0, 10, 3)):
        assert not np.array_equal(a, other)
    # the domain id is folded into the high key word
    assert np.array_equal(normals((1 << 32) * 3, 0, 4, 4), normals(0, 3, 4, 4))
