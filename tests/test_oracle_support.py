"""Pins of the oracle's support-weighted confidence (Sec. 3.1, after Eq. (6); reading R10)
against facts the mathematics fixes: a hand-worked 1 x 3 case in both orientations, the
explicit sum over products of weights on tiny images, closed forms and Toeplitz cascades
for a uniform guide, independence of the two sides of a hard edge, and the range (0, 1]."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import _load_golden


def _line_sum_matrix(w):
    """Unnormalised two-sided kernel of one line, from the explicit products of the
    weights between every pair of samples (pure Python loops)."""
    L = len(w)
    M = np.zeros((L, L))
    for n in range(L):
        for j in range(L):
            p = 1.0
            for k in range(min(n, j) + 1, max(n, j) + 1):
                p *= w[k]
            M[n, j] = p
    return M


def _explicit_support(dx, dy, sigma_s, N):
    H, W = dx.shape
    s = np.ones((H, W))
    for a in oracle.feedback_coefficients(sigma_s, N):
        m = (1.0 - a) / (1.0 + a)
        r = np.empty_like(s)
        for y in range(H):
            r[y] = m * _line_sum_matrix([a ** float(d) for d in dx[y]]) @ s[y]
        c = np.empty_like(r)
        for x in range(W):
            c[:, x] = m * _line_sum_matrix([a ** float(d) for d in dy[:, x]]) @ r[:, x]
        s = c
    return s


def test_support_golden_1x3_both_orientations():
    (ss, s0, s1, s2, q0, q1, q2), = _load_golden("support_1x3.txt")
    for shape, view in (((1, 1, 3), lambda a: a[0]), ((1, 3, 1), lambda a: a[:, 0])):
        guide = np.full(shape, 0.25)
        c, s = oracle.support_confidence(guide, np.full(shape, 0.5), ss, 0.1, filter_iters=1)
        assert np.allclose(view(s), [s0, s1, s2], rtol=0, atol=1e-14)
        assert np.allclose(view(c[0]), [q0, q1, q2], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,N", [(0, 1), (1, 2), (2, 3)])
def test_support_is_the_explicit_sum_over_weight_products(seed, N):
    rng = np.random.default_rng(40 + seed)
    H, W, ss, sr = 5, 7, 5.0, 0.6
    guide = rng.random((2, H, W))
    dx, dy = oracle.distances(guide, ss, sr)
    ref = _explicit_support(dx, dy, ss, N)
    assert np.abs(oracle.support(guide, ss, sr, N) - ref).max() <= 1e-13


def test_uniform_guide_closed_form_one_iteration():
    # one iteration on a uniform guide factorises into per-axis finite geometric sums:
    # S_L[n] = (1 - a^(n+1))/(1 - a) + (1 - a^(L-n))/(1 - a) - 1
    H, W, ss = 37, 53, 6.0
    (a,) = oracle.feedback_coefficients(ss, 1)
    m = (1 - a) / (1 + a)

    def axis(L):
        n = np.arange(L)
        return m * ((1 - a ** (n + 1)) / (1 - a) + (1 - a ** (L - n)) / (1 - a) - 1)

    s = oracle.support(np.zeros((1, H, W)), ss, 0.2, filter_iters=1)
    assert np.abs(s - np.outer(axis(H), axis(W))).max() <= 1e-13
    # far from the borders the support of a flat region is 1; at a corner 1/(1+a)^2
    big = oracle.support(np.zeros((1, 1, 1)), ss, 0.2, filter_iters=1)
    assert abs(big[0, 0] - m * m) <= 1e-15
    assert abs(axis(4001)[2000] - 1.0) <= 1e-12
    assert abs(axis(4001)[0] - 1.0 / (1.0 + a)) <= 1e-12


def test_uniform_guide_three_iterations_is_a_toeplitz_cascade():
    H, W, ss = 23, 31, 8.0
    alist = oracle.feedback_coefficients(ss, 3)

    def axis(L):
        idx = np.arange(L)
        v = np.ones(L)
        for a in alist:
            T = np.power(a, np.abs(idx[:, None] - idx[None, :]).astype(float))
            v = (1 - a) / (1 + a) * (T @ v)
        return v

    s = oracle.support(np.full((3, H, W), 0.6), ss, 0.1)
    assert np.abs(s - np.outer(axis(H), axis(W))).max() <= 1e-13


def test_hard_edge_separates_the_two_sides():
    # a guide step far above sigma_r gives weight a^d = 0 (underflow) across it: the part
    # right of the step has exactly the support of a flat image of its own width
    H, W, c0 = 9, 30, 11
    guide = np.zeros((1, H, W))
    guide[0, :, c0:] = 1.0
    s = oracle.support(guide, 8.0, 1e-6)
    right = oracle.support(np.zeros((1, H, W - c0)), 8.0, 1e-6)
    left = oracle.support(np.zeros((1, H, c0)), 8.0, 1e-6)
    assert np.array_equal(s[:, c0:], right)
    assert np.array_equal(s[:, :c0], left)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_relative_support_lies_in_zero_one(seed):
    # every weight a^d <= a (d >= 1): the support never exceeds a flat region's
    rng = np.random.default_rng(70 + seed)
    guide = rng.random((3, 16, 21)) * rng.uniform(0.01, 1.0)
    s = oracle.support(guide, rng.uniform(2, 20), rng.uniform(0.05, 0.5))
    assert s.min() > 0.0 and s.max() <= 1.0 + 1e-12


def test_weighted_confidence_divides_every_channel():
    rng = np.random.default_rng(3)
    guide = rng.random((3, 6, 8))
    conf = rng.uniform(0.1, 1.0, (2, 6, 8))
    c, s = oracle.support_confidence(guide, conf, 4.0, 0.3)
    assert np.abs(c * s[None] - conf).max() <= 1e-14
