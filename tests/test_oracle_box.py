"""Pins of the oracle's box form of the edge-aware mean (Sec. 3.2, Eq. (10) read literally;
readings B1-B4) against facts the mathematics fixes: the integer codes and radii in closed
form, the truncated moving average of a uniform guide (a library convolution), explicit
membership sums on tiny inputs, invariants (constants, symmetry of the unnormalised
kernel, hard edges), and the solver loop on a uniform guide."""
import math

import numpy as np
import pytest

import oracle


def _moving_average(f, h):
    # normalised convolution with a box of 2h + 1 samples, truncated at the ends
    k = np.ones(2 * h + 1)
    return np.convolve(f, k, mode="same") / np.convolve(np.ones_like(f), k, mode="same")


def test_codes_of_uniform_and_step_guides():
    qx, qy = oracle.box_codes(np.full((3, 5, 7), 0.3, dtype=np.float32), 8.0, 0.2)
    assert np.all(qx[:, 1:] == 256) and np.all(qy[1:, :] == 256)
    # one band with a step of 0.5 between columns 2 and 3: d = sqrt(1 + (8/0.25)^2 0.25)
    g = np.zeros((1, 2, 6), dtype=np.float32)
    g[0, :, 3:] = 0.5
    qx, qy = oracle.box_codes(g, 8.0, 0.25)
    assert list(qx[0]) == [0, 256, 256, round(256 * math.sqrt(1 + 32.0 ** 2 * 0.25)), 256, 256]
    assert np.all(qy[1] == 256)


def test_codes_round_the_fp64_distance():
    rng = np.random.default_rng(3)
    g = rng.random((4, 20, 30)).astype(np.float32)
    qx, qy = oracle.box_codes(g, 6.0, 0.3)
    dx, dy = oracle.distances(g, 6.0, 0.3)
    assert np.abs(qx[:, 1:] - 256 * dx[:, 1:]).max() <= 0.5 + 1e-3
    assert np.abs(qy[1:, :] - 256 * dy[1:, :]).max() <= 0.5 + 1e-3


def test_radii_closed_form():
    # sigma_H1 = 8 sqrt(3) 4 / sqrt(63), r1 = sqrt(3) sigma_H1 = 96 / sqrt(63); r halves
    assert oracle.box_radii(8.0, 3) == [math.floor(256 * 96 / math.sqrt(63)),
                                        math.floor(128 * 96 / math.sqrt(63)),
                                        math.floor(64 * 96 / math.sqrt(63))]
    # one iteration: sigma_H = sigma_s, r = sqrt(3) sigma_s
    assert oracle.box_radii(10.0, 1) == [math.floor(256 * math.sqrt(3) * 10.0)]


@pytest.mark.parametrize("R", [100, 256, 3096, 1548])
def test_uniform_guide_is_a_truncated_moving_average(R):
    rng = np.random.default_rng(R)
    L = 57
    f = rng.random((L, 3))
    q = np.full((L, 3), 256)
    out = oracle.box_lines(f, q, R)
    for m in range(3):
        assert np.abs(out[:, m] - _moving_average(f[:, m], R // 256)).max() <= 1e-13


def test_membership_by_brute_force():
    rng = np.random.default_rng(8)
    L, M, R = 23, 4, 900
    f = rng.random((L, M))
    q = rng.integers(256, 700, size=(L, M))
    out = oracle.box_lines(f, q, R)
    for m in range(M):
        ct = [0]
        for n in range(1, L):
            ct.append(ct[-1] + int(q[n, m]))
        for n in range(L):
            members = [j for j in range(L) if abs(ct[n] - ct[j]) <= R]
            assert abs(out[n, m] - sum(f[j, m] for j in members) / len(members)) <= 1e-14


def test_constant_signal_is_preserved():
    rng = np.random.default_rng(2)
    g = rng.random((3, 17, 19)).astype(np.float32)
    qx, qy = oracle.box_codes(g, 5.0, 0.2)
    z = oracle.box_filter(np.full((2, 17, 19), 0.625), qx, qy, 5.0, 3)
    assert np.abs(z - 0.625).max() <= 1e-15


def test_unnormalised_kernel_is_symmetric():
    # count[n] * out[n] = sum_j [j in box(n)] f[j], and j in box(n) iff n in box(j)
    rng = np.random.default_rng(5)
    L, R = 31, 1200
    q = rng.integers(256, 900, size=(L, 1))
    cnt = oracle.box_lines(np.ones((L, 1)), q, R)[:, 0]
    assert np.all(cnt == 1.0)
    E = np.eye(L)
    A = np.stack([oracle.box_lines(E[:, [j]], q, R)[:, 0] for j in range(L)], axis=1)
    counts = 1.0 / np.array([A[n, n] for n in range(L)])
    K = A * counts[:, None]
    assert np.array_equal(np.rint(K), K) and np.array_equal(K, K.T)


def test_hard_edge_is_not_crossed():
    H, W, c0 = 5, 24, 10
    g = np.zeros((1, H, W), dtype=np.float32)
    g[0, :, c0:] = 1.0
    qx, qy = oracle.box_codes(g, 8.0, 0.01)
    f = np.where(np.arange(W) < c0, 0.2, 0.9)[None, None, :].repeat(H, axis=1)
    z = oracle.box_filter(f, qx, qy, 8.0, 3)
    assert np.abs(z - f).max() <= 1e-15


def test_solver_on_a_uniform_guide():
    # with a uniform guide every pass is a moving average: run the Eq. (3) iteration with
    # library convolutions and compare
    rng = np.random.default_rng(9)
    H, W, ss, T = 21, 33, 6.0, 4
    t = rng.random((1, H, W))
    c = rng.uniform(0.1, 1.0, (1, H, W))
    hs = [R // 256 for R in oracle.box_radii(ss, 3)]

    def box(z):
        for h in hs:
            z = np.stack([_moving_average(z[y], h) for y in range(H)])
            z = np.stack([_moving_average(z[:, x], h) for x in range(W)], axis=1)
        return z

    z = t[0].copy()
    for _ in range(T):
        z = z - 0.99 * (0.99 * (z - box(z)) + c[0] * (z - t[0]))
    got = oracle.solve_box(np.zeros((1, H, W), dtype=np.float32), t, c, ss, 0.2, 3, T)
    assert np.abs(got[0] - z).max() <= 1e-13
