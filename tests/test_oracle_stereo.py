"""Pins of the oracle's stereo refinement (Sec. 3.3, Eq. (11), readings S1-S5) against facts
the paper and the mathematics fix: linear interpolation closed forms, finite differences
of the Eq. (11) energy, a pair related by an exact shift, the L1 limit of the Charbonnier
loss, and the reduction to the plain solver when the photometric term is off."""
import numpy as np
import pytest

import oracle


def test_row_sampling_closed_forms():
    img = np.array([[[0.0, 1.0, 4.0, 9.0, 16.0]]])  # x^2 on one row
    xs = np.array([[0.0, 2.0, 4.0, 2.5, 0.25, -3.0, 7.0, 3.999]])
    v, s = oracle.sample_row_linear(img, xs)
    assert np.allclose(v[0, 0], [0.0, 4.0, 16.0, 6.5, 0.25, 0.0, 16.0, 16.0 - 7 * 0.001])
    # slope of the segment the sample falls in; 0 where the position was clamped
    assert np.allclose(s[0, 0], [1.0, 5.0, 7.0, 5.0, 1.0, 0.0, 0.0, 7.0])
    v1, s1 = oracle.sample_row_linear(np.full((2, 3, 1), 0.3), np.full((3, 1), 5.0))
    assert np.all(v1 == 0.3) and np.all(s1 == 0.0)


def _pair(seed, H=6, W=40, C=3):
    rng = np.random.default_rng(seed)
    left = rng.random((C, H, W))
    right = rng.random((C, H, W))
    # disparities with fractional parts inside (0.2, 0.8): +-h stays on one segment
    z = (rng.integers(0, 8, size=(1, H, W)) + rng.uniform(0.2, 0.8, size=(1, H, W)))
    t = z + rng.normal(0, 0.5, size=z.shape)
    c = rng.uniform(0.1, 1.0, size=z.shape)
    return left, right, z, t, c


@pytest.mark.parametrize("seed", [0, 1])
def test_data_gradient_is_the_energy_derivative(seed):
    left, right, z, t, c = _pair(seed)
    gamma, eps, h = 0.3, 0.05, 1e-6
    D = oracle.stereo_data_gradient(left, right, z, t, c, gamma, eps)
    zbar = np.zeros_like(z)
    fd = np.empty_like(z)
    for idx in np.ndindex(z.shape):
        zp = z.copy(); zp[idx] += h
        zm = z.copy(); zm[idx] -= h
        fd[idx] = (oracle.energy_stereo(zp, zbar, left, right, t, c, 0.0, gamma, eps)
                   - oracle.energy_stereo(zm, zbar, left, right, t, c, 0.0, gamma, eps)) / (2 * h)
    assert np.abs(D - fd).max() <= 1e-6


def test_update_direction_is_the_gradient_with_frozen_mean():
    left, right, z, t, c = _pair(5, H=4, W=24)
    lam, gamma, eps, h = 0.99, 0.01, 0.001, 1e-6
    zbar = z + np.random.default_rng(9).normal(0, 1, size=z.shape)
    g = lam * (z - zbar) + oracle.stereo_data_gradient(left, right, z, t, c, gamma, eps)
    for idx in [(0, 0, 3), (0, 2, 11), (0, 3, 20)]:
        zp = z.copy(); zp[idx] += h
        zm = z.copy(); zm[idx] -= h
        fd = (oracle.energy_stereo(zp, zbar, left, right, t, c, lam, gamma, eps)
              - oracle.energy_stereo(zm, zbar, left, right, t, c, lam, gamma, eps)) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-5 * max(1.0, abs(fd))


def test_exact_shift_has_no_photometric_gradient_at_the_true_disparity():
    rng = np.random.default_rng(4)
    C, H, W, d0 = 3, 5, 30, 4
    right = rng.random((C, H, W))
    left = np.zeros_like(right)
    left[:, :, d0:] = right[:, :, :W - d0]  # I_L(x) = I_R(x - d0)
    z = np.full((1, H, W), float(d0))
    D = oracle.stereo_data_gradient(left, right, z, z, np.zeros_like(z), 1.0, 0.001)
    assert np.abs(D[0, :, d0:]).max() <= 1e-12


def test_tiny_epsilon_gives_the_l1_direction():
    left, right, z, t, c = _pair(7)
    D = oracle.stereo_data_gradient(left, right, z, t, c, 0.0, 1e-12)
    assert np.allclose(D, c * np.sign(z - t), atol=1e-9)


def test_no_photometric_term_and_huge_epsilon_reduce_to_the_plain_solver():
    # rho'(r) = r / sqrt(r^2 + E^2) = (r / E)(1 + O(r^2 / E^2)): the update becomes Eq. (3)
    # with confidence c / E
    rng = np.random.default_rng(11)
    H, W, E = 12, 17, 1e4
    left = rng.random((3, H, W))
    t = rng.random((1, H, W)) * 10
    c = rng.uniform(0.1, 1.0, (1, H, W))
    zs = oracle.solve_stereo(left, rng.random((3, H, W)), t, c, 6.0, 0.2, 3, 5, gamma=0.0, eps=E)
    zp = oracle.solve(left, t, c / E, 6.0, 0.2, 3, 5)
    assert np.abs(zs - zp).max() <= 1e-9
