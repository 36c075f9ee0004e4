"""Pins of the oracle's variance-based confidence (Eq. (7), Sec. 3.1) against facts the
paper and the mathematics fix: a hand-worked 1 x 2 case, constant inputs, Jensen's
inequality, the weighted-variance identity on an independently built filter matrix,
and region-aligned inputs behind a hard guide edge."""
import math
import os

import numpy as np
import pytest

import oracle
from test_oracle_pins import GOLDEN, _load_golden, explicit_dt_matrix


def test_variance_confidence_golden_1x2():
    (ss, sr, sc, v0, v1, c0, c1), = _load_golden("variance_confidence_1x2.txt")
    guide = np.full((1, 1, 2), 0.5)
    z = np.array([[[0.0, 1.0]]])
    c, V = oracle.variance_confidence(guide, z, ss, sr, sc, filter_iters=1)
    assert np.allclose(V[0, 0], [v0, v1], rtol=0, atol=1e-12)
    assert np.allclose(c[0, 0], [c0, c1], rtol=0, atol=1e-12)


def test_constant_input_has_unit_confidence():
    rng = np.random.default_rng(5)
    guide = rng.random((3, 17, 23))
    z = np.stack([np.full((17, 23), 0.3), np.full((17, 23), 0.9)])
    c, V = oracle.variance_confidence(guide, z, 6.0, 0.2, 0.05)
    assert np.abs(V).max() <= 1e-12
    assert np.abs(c - 1.0).max() <= 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_variance_is_nonnegative(seed):
    # DT is a convex combination per pixel (nonnegative weights summing to one), so by
    # Jensen's inequality DT(z^2) >= DT(z)^2
    rng = np.random.default_rng(100 + seed)
    guide = rng.random((2, 19, 13))
    z = rng.random((2, 19, 13)) * 3.0 - 1.0
    c, V = oracle.variance_confidence(guide, z, 5.0, 0.3, 0.5)
    assert V.min() >= -1e-12
    assert c.max() <= 1.0 + 1e-12


def test_variance_equals_weighted_variance_of_explicit_filter():
    # with m = A z and rows of A summing to one:  V_i = sum_j A_ij (z_j - m_i)^2
    rng = np.random.default_rng(7)
    H, W, ss, sr, N = 4, 5, 4.0, 0.25, 2
    guide = rng.random((2, H, W))
    z = rng.random((1, H, W))
    dx, dy = oracle.distances(guide, ss, sr)
    A = explicit_dt_matrix(dx, dy, oracle.feedback_coefficients(ss, N))
    zf = z.ravel()
    m = A @ zf
    V_ref = np.array([np.sum(A[i] * (zf - m[i]) ** 2) for i in range(H * W)])
    c, V = oracle.variance_confidence(guide, z, ss, sr, 0.3, filter_iters=N)
    assert np.abs(V.ravel() - V_ref).max() <= 1e-12
    assert np.abs(c.ravel() - np.exp(-V_ref / (2 * 0.3 ** 2))).max() <= 1e-12


def test_hard_guide_edge_keeps_regions_apart():
    # a guide step far above sigma_r makes every weight across it a^d ~ 0: each side is a
    # separate region, z constant on each side has zero variance, while the same z under a
    # uniform guide mixes the two sides near the step
    H, W = 6, 10
    guide = np.zeros((1, H, W))
    guide[0, :, W // 2:] = 1.0
    z = np.where(np.arange(W) < W // 2, 0.2, 0.8)[None, None, :].repeat(H, axis=1)
    c, V = oracle.variance_confidence(guide, z, 8.0, 1e-3, 0.1)
    assert np.abs(V).max() <= 1e-12
    assert np.abs(c - 1.0).max() <= 1e-10
    c_u, V_u = oracle.variance_confidence(np.zeros((1, H, W)), z, 8.0, 1e-3, 0.1)
    assert V_u[0, :, W // 2 - 1].min() > 1e-3 and c_u.min() < 0.9
