"""Pins of the FP64 oracle against what the paper and plain mathematics fix.

Every test here runs on the CPU.  None of them re-types an oracle formula: each compares
the oracle with an independent route to the same value (a closed form, an explicit sum
written as loops, a dense linear-algebra identity, a special case the paper states, or a
property any correct implementation must have), chosen so that a dropped term, a wrong
sign or index, or a swapped axis in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import dts_inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------
# helpers written independently of the oracle (pure Python loops)
# ---------------------------------------------------------------------------------------
def explicit_pass_matrix(w):
    """Matrix M of one causal+anticausal pass on a line, from the explicit weighted sums

        J[j] = sum_{k<=j} u_k prod_{m=k+1..j} w_m f[k],   u_0 = 1, u_k = 1 - w_k
        K[n] = sum_{j>=n} v_j prod_{m=n+1..j} w_m J[j],   v_{L-1} = 1, v_j = 1 - w_{j+1}

    i.e. M[n, k] = sum_{j >= max(n, k)} v_j prod_{m=n+1..j} w_m u_k prod_{m=k+1..j} w_m."""
    L = len(w)
    M = [[0.0] * L for _ in range(L)]
    for n in range(L):
        for k in range(L):
            total = 0.0
            for j in range(max(n, k), L):
                v = 1.0 if j == L - 1 else 1.0 - w[j + 1]
                u = 1.0 if k == 0 else 1.0 - w[k]
                p1 = 1.0
                for m in range(n + 1, j + 1):
                    p1 *= w[m]
                p2 = 1.0
                for m in range(k + 1, j + 1):
                    p2 *= w[m]
                total += v * p1 * u * p2
            M[n][k] = total
    return np.array(M)


def explicit_dt_matrix(dx, dy, a_list):
    """Dense 2-D filter built from explicit pass matrices: for each filter iteration, every
    row gets its own explicit matrix (weights a^dx of that row), then every column."""
    H, W = dx.shape
    n = H * W
    A = np.eye(n)
    for a in a_list:
        R = np.zeros((n, n))
        for y in range(H):
            M = explicit_pass_matrix([a ** float(d) for d in dx[y]])
            idx = [y * W + x for x in range(W)]
            R[np.ix_(idx, idx)] = M
        C = np.zeros((n, n))
        for x in range(W):
            M = explicit_pass_matrix([a ** float(d) for d in dy[:, x]])
            idx = [y * W + x for y in range(H)]
            C[np.ix_(idx, idx)] = M
        A = C @ R @ A
    return A


# ---------------------------------------------------------------------------------------
# P1: distances (Sec. 3.2, Eq. (8)-(9))
# ---------------------------------------------------------------------------------------
def test_uniform_guide_gives_unit_distances():
    g = np.full((3, 7, 9), 0.37, dtype=np.float32)
    dx, dy = oracle.distances(g, 8.0, 0.2)
    assert np.array_equal(dx, np.ones_like(dx))
    assert np.array_equal(dy, np.ones_like(dy))


def test_step_edge_distance_is_hypotenuse():
    # one channel with a step of height D between columns 3 and 4: the arc length of that
    # step in [x, I*sigma_s/sigma_r] space is sqrt(1 + (s D)^2); elsewhere 1
    s_s, s_r, D = 8.0, 0.2, 0.25
    g = np.zeros((2, 5, 8))
    g[0, :, 4:] = D
    dx, dy = oracle.distances(g, s_s, s_r)
    expect = np.ones((5, 8))
    expect[:, 4] = math.hypot(1.0, s_s / s_r * D)
    np.testing.assert_allclose(dx, expect, rtol=0, atol=1e-13)
    assert np.array_equal(dy, np.ones_like(dy))


def test_distance_uses_l2_norm_across_channels():
    # two channels stepping by 0.3 and 0.4 at the same column: ||(0.3, 0.4)|| = 0.5
    g = np.zeros((2, 4, 6))
    g[0, :, 3:] = 0.3
    g[1, :, 3:] = 0.4
    dx, _ = oracle.distances(g, 1.0, 1.0)
    np.testing.assert_allclose(dx[:, 3], math.hypot(1.0, 0.5), atol=1e-14)


def test_linear_ramp_has_constant_arc_length():
    # I(x) = g x has arc-length element sqrt(1 + (s g)^2) everywhere (integral of Eq. (9))
    gslope, s_s, s_r = 0.01, 16.0, 0.1
    ramp = gslope * np.arange(11, dtype=np.float64)
    g = np.broadcast_to(ramp, (1, 5, 11)).copy()
    dx, dy = oracle.distances(g, s_s, s_r)
    np.testing.assert_allclose(dx[:, 1:], math.sqrt(1 + (s_s / s_r * gslope) ** 2), rtol=1e-13)
    assert np.array_equal(dy, np.ones_like(dy))


def test_dy_is_dx_of_transposed_guide():
    rng = np.random.default_rng(5)
    g = rng.uniform(size=(3, 6, 9))
    dx, dy = oracle.distances(g, 5.0, 0.3)
    dxT, dyT = oracle.distances(g.transpose(0, 2, 1), 5.0, 0.3)
    np.testing.assert_array_equal(dy, dxT.T)
    np.testing.assert_array_equal(dx, dyT.T)


def test_distances_accept_band_iterator():
    rng = np.random.default_rng(6)
    g = rng.uniform(size=(4, 5, 7)).astype(np.float32)
    a = oracle.distances(g, 6.0, 0.2)
    b = oracle.distances(iter(list(g)), 6.0, 0.2)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ---------------------------------------------------------------------------------------
# P2: one 1-D pass (recursive filter)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 3, 7, 16])
def test_pass_equals_explicit_weighted_sum(L):
    rng = np.random.default_rng(L)
    w = rng.uniform(0.0, 1.0, size=L)
    f = rng.normal(size=L)
    M = explicit_pass_matrix(list(w))
    K = oracle.rf1d_lines(f, w)
    np.testing.assert_allclose(K, M @ f, rtol=0, atol=1e-14)


def test_pass_matrix_is_row_stochastic_and_nonnegative():
    rng = np.random.default_rng(11)
    L = 12
    w = rng.uniform(0.0, 1.0, size=L)
    cols = [oracle.rf1d_lines(np.eye(L)[:, j], w) for j in range(L)]
    M = np.stack(cols, axis=1)
    assert M.min() >= 0.0
    np.testing.assert_allclose(M.sum(axis=1), 1.0, atol=1e-15)


def test_pass_preserves_constants_and_range():
    rng = np.random.default_rng(12)
    w = rng.uniform(0.0, 1.0, size=(50, 8))
    K = oracle.rf1d_lines(np.full((50, 8), 0.731), w)
    np.testing.assert_allclose(K, 0.731, atol=1e-15)
    f = rng.uniform(-2.0, 3.0, size=(50, 8))
    K = oracle.rf1d_lines(f, w)
    assert K.min() >= f.min(axis=0).min() - 1e-15
    assert np.all(K.max(axis=0) <= f.max(axis=0) + 1e-15)
    assert np.all(K.min(axis=0) >= f.min(axis=0) - 1e-15)


def test_zero_weights_are_identity():
    f = np.random.default_rng(13).normal(size=(9, 3))
    np.testing.assert_array_equal(oracle.rf1d_lines(f, np.zeros((9, 3))), f)


def test_uniform_weight_closed_form():
    # w == a: J[n] = a^n f[0] + (1-a) sum_{k=1..n} a^(n-k) f[k], and the mirrored form for K
    a, L = 0.8, 20
    f = np.random.default_rng(14).normal(size=L)
    J = np.array([a ** n * f[0] + (1 - a) * sum(a ** (n - k) * f[k] for k in range(1, n + 1))
                  for n in range(L)])
    K = np.array([a ** (L - 1 - n) * J[L - 1]
                  + (1 - a) * sum(a ** (j - n) * J[j] for j in range(n, L - 1))
                  for n in range(L)])
    Ko, Jo = oracle.rf1d_lines(f, np.full(L, a), return_intermediates=True)
    np.testing.assert_allclose(Jo, J, atol=1e-14)
    np.testing.assert_allclose(Ko, K, atol=1e-14)


# ---------------------------------------------------------------------------------------
# P3: filter schedule and the uniform-guide closed forms
# ---------------------------------------------------------------------------------------
def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


def test_schedule_matches_golden_fractions():
    # sigma_Hi / sigma_s for N = 3 is sqrt(3 * 4^(N-i) / (4^N - 1)) = sqrt(48/63), sqrt(12/63),
    # sqrt(3/63); the fixture holds these ratios and a = exp(-sqrt(2)/sigma_H) at sigma_s = 8, 32
    rows = _load_golden("schedule_n3.txt")
    for sigma_s, r1, r2, r3, a1, a2, a3 in rows:
        a = oracle.feedback_coefficients(sigma_s, 3)
        sig = [-math.sqrt(2.0) / math.log(x) for x in a]
        np.testing.assert_allclose(np.array(sig) / sigma_s, [r1, r2, r3], rtol=1e-12)
        np.testing.assert_allclose(a, [a1, a2, a3], rtol=1e-12)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_schedule_variances_sum_to_sigma_s_squared(N):
    sigma_s = 13.0
    a = oracle.feedback_coefficients(sigma_s, N)
    sig2 = sum((math.sqrt(2.0) / math.log(x)) ** 2 for x in a)
    assert abs(sig2 - sigma_s ** 2) < 1e-9
    # successive sigma_H halve
    sig = [-math.sqrt(2.0) / math.log(x) for x in a]
    for i in range(1, N):
        assert abs(sig[i - 1] / sig[i] - 2.0) < 1e-12


def test_impulse_variance_closed_form_1d():
    # a 1 x L image under a uniform guide is the 1-D filter; a one-sided geometric kernel
    # (1-a) a^k has variance a/(1-a)^2, causal+anticausal doubles it, iterations add up
    L, x0, sigma_s = 2001, 1000, 8.0
    g = np.zeros((1, 1, L))
    dx, dy = oracle.distances(g, sigma_s, 1.0)
    e = np.zeros((1, 1, L))
    e[0, 0, x0] = 1.0
    h = oracle.dt_filter(e, dx, dy, sigma_s, 3)[0, 0]
    x = np.arange(L) - x0
    a = oracle.feedback_coefficients(sigma_s, 3)
    assert abs(h.sum() - 1.0) < 1e-12
    assert abs((h * x).sum()) < 1e-9                         # symmetric about the impulse
    var = (h * x * x).sum()
    expect = sum(2 * ai / (1 - ai) ** 2 for ai in a)
    assert abs(var - expect) < 1e-8 * expect
    assert abs(var - sigma_s ** 2) < 0.05 * sigma_s ** 2     # continuum limit: sigma_s^2


def test_uniform_guide_2d_is_separable_even_at_borders():
    # with a uniform guide every row uses the same weights and every column too, so row
    # and column passes commute and the 2-D impulse response is the outer product of the
    # 1-D responses, border effects included
    H, W, sigma_s = 13, 17, 3.0
    g = np.zeros((1, H, W))
    dx, dy = oracle.distances(g, sigma_s, 1.0)
    for (y0, x0) in [(0, 0), (6, 8), (12, 3)]:
        e = np.zeros((1, H, W))
        e[0, y0, x0] = 1.0
        h2 = oracle.dt_filter(e, dx, dy, sigma_s, 3)[0]
        er = np.zeros((1, 1, W))
        er[0, 0, x0] = 1.0
        hr = oracle.dt_filter(er, dx[:1], dy[:1], sigma_s, 3)[0, 0]
        ec = np.zeros((1, 1, H))
        ec[0, 0, y0] = 1.0
        hc = oracle.dt_filter(ec, np.ones((1, H)), np.ones((1, H)), sigma_s, 3)[0, 0]
        np.testing.assert_allclose(h2, np.outer(hc, hr), atol=1e-15)


def test_dt_equals_explicit_pass_composition():
    # the whole 2-D filter (three iterations of rows-then-columns with a^dx, a^dy) against
    # a dense product of explicitly summed pass matrices, on a random 4x5 guide
    rng = np.random.default_rng(21)
    g = rng.uniform(size=(2, 4, 5))
    sigma_s, sigma_r = 3.0, 0.5
    dx, dy = oracle.distances(g, sigma_s, sigma_r)
    a = oracle.feedback_coefficients(sigma_s, 3)
    A_explicit = explicit_dt_matrix(dx, dy, a)
    A = oracle.dense_filter_matrix(dx, dy, sigma_s, 3)
    np.testing.assert_allclose(A, A_explicit, atol=1e-14)
    # and the order matters: columns-then-rows gives a different matrix on this guide
    A_swapped = explicit_dt_matrix(dy.T.copy(), dx.T.copy(), a)
    P = np.zeros((20, 20))
    for y in range(4):
        for x in range(5):
            P[y * 5 + x, x * 4 + y] = 1.0
    assert np.abs(P @ A_swapped @ P.T - A).max() > 1e-6


# ---------------------------------------------------------------------------------------
# P4: a hard edge cuts the filter
# ---------------------------------------------------------------------------------------
def test_hard_edge_splits_the_image():
    rng = np.random.default_rng(31)
    H, W, x0 = 9, 14, 6
    g = np.zeros((1, H, W))
    g[0, :, x0:] = 1.0
    sigma_s, sigma_r = 4.0, 1e-9          # a^d underflows to exactly 0 across the edge
    z = rng.normal(size=(2, H, W))
    dx, dy = oracle.distances(g, sigma_s, sigma_r)
    full = oracle.dt_filter(z, dx, dy, sigma_s, 3)
    for sl in (slice(0, x0), slice(x0, W)):
        dxs, dys = oracle.distances(g[:, :, sl], sigma_s, sigma_r)
        part = oracle.dt_filter(z[:, :, sl], dxs, dys, sigma_s, 3)
        np.testing.assert_array_equal(full[:, :, sl], part)


# ---------------------------------------------------------------------------------------
# P5: structure of the 2-D filter
# ---------------------------------------------------------------------------------------
def test_dt_is_linear_and_channel_independent():
    rng = np.random.default_rng(41)
    g = rng.uniform(size=(3, 10, 11))
    dx, dy = oracle.distances(g, 5.0, 0.2)
    p = rng.normal(size=(1, 10, 11))
    q = rng.normal(size=(1, 10, 11))
    lhs = oracle.dt_filter(2.5 * p - 0.75 * q, dx, dy, 5.0, 3)
    rhs = 2.5 * oracle.dt_filter(p, dx, dy, 5.0, 3) - 0.75 * oracle.dt_filter(q, dx, dy, 5.0, 3)
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
    both = oracle.dt_filter(np.concatenate([p, q]), dx, dy, 5.0, 3)
    np.testing.assert_array_equal(both[0], oracle.dt_filter(p, dx, dy, 5.0, 3)[0])
    np.testing.assert_array_equal(both[1], oracle.dt_filter(q, dx, dy, 5.0, 3)[0])


def test_dense_filter_is_stochastic_with_unit_spectral_radius():
    rng = np.random.default_rng(42)
    g = rng.uniform(size=(3, 8, 9))
    dx, dy = oracle.distances(g, 4.0, 0.3)
    A = oracle.dense_filter_matrix(dx, dy, 4.0, 3)
    assert A.min() >= 0.0
    np.testing.assert_allclose(A.sum(axis=1), 1.0, atol=1e-14)
    ev = np.linalg.eigvals(A)
    assert abs(np.abs(ev).max() - 1.0) < 1e-10
    # A is not symmetric on a non-uniform guide (so no test may assume symmetry)
    assert np.abs(A - A.T).max() > 1e-3


# ---------------------------------------------------------------------------------------
# P6-P7: special cases and the dense form of the solver (Sec. 3.1, Eq. (3)-(4))
# ---------------------------------------------------------------------------------------
def _tiny(seed, H=6, W=7, Cg=2, Ct=1):
    rng = np.random.default_rng(seed)
    g = rng.uniform(size=(Cg, H, W))
    t = rng.uniform(size=(Ct, H, W))
    c = rng.uniform(0.1, 1.0, size=(Ct, H, W))
    return g, t, c


def test_zero_iterations_return_target():
    g, t, c = _tiny(51)
    np.testing.assert_array_equal(oracle.solve(g, t, c, 4.0, 0.2, 3, 0), t)


def test_constant_target_is_a_fixed_point():
    g, _, c = _tiny(52)
    t = np.full((1, 6, 7), 0.42)
    np.testing.assert_allclose(oracle.solve(g, t, c, 4.0, 0.2, 3, 7), t, atol=1e-15)


def test_zero_confidence_one_step_is_dt_blend():
    # the paper notes that zero confidence reduces the solver to domain-transform filtering
    g, t, _ = _tiny(53)
    c = np.zeros_like(t)
    lam, step = 0.99, 0.99
    dx, dy = oracle.distances(g, 4.0, 0.2)
    A = oracle.dense_filter_matrix(dx, dy, 4.0, 3)
    z1 = oracle.solve(g, t, c, 4.0, 0.2, 3, 1, lam, step)
    expect = (1 - step * lam) * t.ravel() + step * lam * (A @ t.ravel())
    np.testing.assert_allclose(z1.ravel(), expect, atol=1e-14)
    T = 6
    zT = oracle.solve(g, t, c, 4.0, 0.2, 3, T, lam, step)
    Pm = np.linalg.matrix_power((1 - step * lam) * np.eye(42) + step * lam * A, T)
    np.testing.assert_allclose(zT.ravel(), Pm @ t.ravel(), atol=1e-13)


def test_solver_matches_dense_affine_recursion():
    g, t, c = _tiny(54)
    lam, step, T = 0.99, 0.99, 5
    dx, dy = oracle.distances(g, 4.0, 0.2)
    A = oracle.dense_filter_matrix(dx, dy, 4.0, 3)
    C = np.diag(c.ravel())
    P = np.eye(42) - step * (lam * (np.eye(42) - A) + C)
    expect = np.linalg.matrix_power(P, T) @ t.ravel()
    for j in range(T):
        expect = expect + np.linalg.matrix_power(P, j) @ (step * C @ t.ravel())
    z = oracle.solve(g, t, c, 4.0, 0.2, 3, T, lam, step)
    np.testing.assert_allclose(z.ravel(), expect, atol=1e-13)


def test_long_run_reaches_eq4_stationary_point():
    g, t, c = _tiny(55, H=5, W=6)
    lam, step = 0.99, 0.99
    dx, dy = oracle.distances(g, 4.0, 0.2)
    A = oracle.dense_filter_matrix(dx, dy, 4.0, 3)
    C = np.diag(c.ravel())
    zstar = np.linalg.solve(lam * (np.eye(30) - A) + C, C @ t.ravel())
    z = oracle.solve(g, t, c, 4.0, 0.2, 3, 3000, lam, step)
    np.testing.assert_allclose(z.ravel(), zstar, atol=1e-12)
    # Eq. (4): z_i = (lam * zbar_i + c_i t_i) / (lam + c_i) at the stationary point
    zbar = oracle.dt_filter(z, dx, dy, 4.0, 3)
    np.testing.assert_allclose(z, (lam * zbar + c * t) / (lam + c), atol=1e-12)


def test_broadcast_confidence_equals_repeated_channels():
    g, t, c = _tiny(56, Ct=3)
    c1 = c[:1]
    a = oracle.solve(g, t, c1, 4.0, 0.2, 3, 4)
    b = oracle.solve(g, t, np.repeat(c1, 3, axis=0), 4.0, 0.2, 3, 4)
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------------------------------
# P8: dynamics over the solver iterations on the 256x256 polygon and 1920x1080 disparity workloads
# ---------------------------------------------------------------------------------------
def _energy_and_residual_trace(case):
    dx, dy = oracle.distances(case["guide"], case["sigma_s"], case["sigma_r"])
    _, its = oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"],
                          case["sigma_r"], case["filter_iters"], case["solver_iters"],
                          case["lam"], case["step"], return_iterates=True, dists=(dx, dy))
    E, R2, Rinf = [], [], []
    for z in its:
        E.append(oracle.energy_e2(z, case["target"], case["conf"], dx, dy, case["sigma_s"],
                                  case["filter_iters"], case["lam"]))
        r = oracle.residual(z, case["target"], case["conf"], dx, dy, case["sigma_s"],
                            case["filter_iters"], case["lam"])
        R2.append(np.sqrt(np.sum(r * r)))
        Rinf.append(np.abs(r).max())
    return np.array(E), np.array(R2), np.array(Rinf)


def test_energy_and_residual_fall_monotonically_polygon_256():
    E, R2, _ = _energy_and_residual_trace(dts_inputs.polygon_256())
    assert np.all(np.diff(E) <= 1e-12 * E[0]), E
    assert np.all(np.diff(R2) <= 1e-12 * R2[0]), R2
    assert E[-1] < 0.5 * E[0]


def test_energy_and_residual_on_disparity_1920x1080():
    # The Eq. (3) direction drops dDT/dz and the filter matrix is not symmetric, so the
    # update is not an exact gradient of E2: on this workload E2 falls for the first 15
    # iterations and then wobbles by < 1e-4 relative, while the L2 norm of the Eq. (3)
    # residual keeps falling at every iteration.
    E, R2, _ = _energy_and_residual_trace(dts_inputs.disparity_1920x1080())
    assert np.all(np.diff(E[:16]) <= 1e-12 * E[0]), E
    assert np.all(np.diff(E) <= 1e-4 * E[-1]), E
    assert np.all(np.diff(R2) <= 1e-12 * R2[0]), R2
    assert E[-1] < 0.1 * E[0]


# The two diagnostics of reading R6, pinned to the explicitly summed filter matrix (built
# above from pure-Python pass matrices, independently of the oracle's filter) and to
# each other.  With A that matrix and C = diag(c):
#   E2(z) = lam/2 |(I - A) z|^2 + 1/2 (z - t)^T C (z - t),
#   grad E2 = lam (I - A)^T (I - A) z + C (z - t),
#   residual(z) = lam (I - A) z + C (z - t)  (the Eq. (3) direction: grad E2 with DT(z)
#   held fixed), so grad E2 = residual - lam A^T (I - A) z.
def _energy_case(seed, H=4, W=5):
    g, t, c = _tiny(seed, H=H, W=W)
    s_s, s_r = 3.0, 0.3
    dx, dy = oracle.distances(g, s_s, s_r)
    A = explicit_dt_matrix(dx, dy, oracle.feedback_coefficients(s_s, 3))
    z = np.random.default_rng(seed + 1000).uniform(size=t.shape)
    return g, t, c, dx, dy, s_s, A, z


def test_energy_e2_matches_dense_closed_form():
    _, t, c, dx, dy, s_s, A, z = _energy_case(71)
    lam = 0.99
    n = A.shape[0]
    v = (np.eye(n) - A) @ z.ravel()
    d = (z - t).ravel()
    closed = 0.5 * lam * float(v @ v) + 0.5 * float(d @ (c.ravel() * d))
    e = oracle.energy_e2(z, t, c, dx, dy, s_s, 3, lam)
    assert abs(e - closed) <= 1e-13 * closed, (e, closed)


def test_residual_matches_dense_closed_form():
    _, t, c, dx, dy, s_s, A, z = _energy_case(72)
    lam = 0.99
    n = A.shape[0]
    closed = lam * (np.eye(n) - A) @ z.ravel() + c.ravel() * (z - t).ravel()
    r = oracle.residual(z, t, c, dx, dy, s_s, 3, lam)
    np.testing.assert_allclose(r.ravel(), closed, atol=1e-14)


def test_energy_gradient_is_residual_plus_the_frozen_filter_term():
    # Central differences of E2 (a quadratic, so exact up to rounding) against the
    # residual: they differ exactly by the derivative of DT(z), which the Eq. (3)
    # direction leaves out.  A lam/2-for-lam slip in E2, a sign in either function or a
    # transposed A fails this.
    _, t, c, dx, dy, s_s, A, z = _energy_case(73)
    lam = 0.99
    n = A.shape[0]
    r = oracle.residual(z, t, c, dx, dy, s_s, 3, lam).ravel()
    frozen_term = lam * A.T @ ((np.eye(n) - A) @ z.ravel())
    h = 1e-4
    for j in range(n):
        zp, zm = z.copy(), z.copy()
        zp.flat[j] += h
        zm.flat[j] -= h
        fd = (oracle.energy_e2(zp, t, c, dx, dy, s_s, 3, lam)
              - oracle.energy_e2(zm, t, c, dx, dy, s_s, 3, lam)) / (2 * h)
        assert abs(fd - (r[j] - frozen_term[j])) <= 1e-9, (j, fd, r[j] - frozen_term[j])


def test_residual_vanishes_at_the_eq4_solution_and_drives_one_step():
    # Eq. (4): at the solution of (lam (I - A) + C) z = C t the Eq. (3) direction is zero;
    # and one descent step from the target is t - step * residual(t).
    g, t, c, dx, dy, s_s, A, _ = _energy_case(74)
    lam, step = 0.99, 0.99
    n = A.shape[0]
    zstar = np.linalg.solve(lam * (np.eye(n) - A) + np.diag(c.ravel()), c.ravel() * t.ravel())
    r = oracle.residual(zstar.reshape(t.shape), t, c, dx, dy, s_s, 3, lam)
    assert np.abs(r).max() <= 1e-13
    assert np.abs(oracle.residual(t, t, c, dx, dy, s_s, 3, lam)).max() > 1e-3
    z1 = oracle.solve(g, t, c, s_s, 0.3, 3, 1, lam, step)
    np.testing.assert_allclose(z1, t - step * oracle.residual(t, t, c, dx, dy, s_s, 3, lam), atol=1e-15)


def test_energy_is_zero_at_a_constant_fixed_point():
    g, _, c, dx, dy, s_s, _, _ = _energy_case(75)
    t = np.full((1,) + dx.shape, 0.42)
    assert oracle.energy_e2(t, t, c, dx, dy, s_s, 3) <= 1e-28
    assert np.abs(oracle.residual(t, t, c, dx, dy, s_s, 3)).max() <= 1e-15


# ---------------------------------------------------------------------------------------
# P9: adjoint against central finite differences and the dense Jacobian
# ---------------------------------------------------------------------------------------
def _loss(g, t, c, ref, s_s, s_r, T):
    z = oracle.solve(g, t, c, s_s, s_r, 3, T)
    return float(np.sum((z - ref) ** 2))


@pytest.mark.parametrize("Cc", [2, 1])
def test_adjoint_matches_central_differences(Cc):
    rng = np.random.default_rng(61)
    H, W, Cg, Ct, T = 7, 6, 2, 2, 3
    s_s, s_r = 3.0, 0.4
    g = rng.uniform(size=(Cg, H, W))
    t = rng.uniform(size=(Ct, H, W))
    c = rng.uniform(0.1, 1.0, size=(Cc, H, W))
    ref = rng.uniform(size=(Ct, H, W))
    z = oracle.solve(g, t, c, s_s, s_r, 3, T)
    gt, gc, gg = oracle.solve_backward(g, t, c, s_s, s_r, 2 * (z - ref), 3, T)
    assert gt.shape == t.shape and gc.shape == c.shape and gg.shape == g.shape
    for name, arr, grad in (("t", t, gt), ("c", c, gc), ("g", g, gg)):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            args = {"t": t, "c": c, "g": g}
            plus = {k: v.copy() for k, v in args.items()}
            minus = {k: v.copy() for k, v in args.items()}
            plus[name][idx] += h
            minus[name][idx] -= h
            fd = (_loss(plus["g"], plus["t"], plus["c"], ref, s_s, s_r, T)
                  - _loss(minus["g"], minus["t"], minus["c"], ref, s_s, s_r, T)) / (2 * h)
            scale = max(abs(fd), 1e-3 * np.abs(grad).max())
            assert abs(grad[idx] - fd) <= 1e-6 * scale, (name, idx, grad[idx], fd)


def test_adjoint_target_gradient_equals_dense_jacobian():
    # dz^T/dt = P^T + sum_{j<T} P^j step C with P = I - step (lam (I - A) + C)
    g, t, c = _tiny(62)
    lam, step, T = 0.99, 0.99, 4
    dx, dy = oracle.distances(g, 4.0, 0.2)
    A = oracle.dense_filter_matrix(dx, dy, 4.0, 3)
    C = np.diag(c.ravel())
    n = A.shape[0]
    P = np.eye(n) - step * (lam * (np.eye(n) - A) + C)
    Jm = np.linalg.matrix_power(P, T)
    for j in range(T):
        Jm = Jm + np.linalg.matrix_power(P, j) @ (step * C)
    go = np.random.default_rng(63).normal(size=t.shape)
    gt, _, _ = oracle.solve_backward(g, t, c, 4.0, 0.2, go, 3, T, lam, step)
    np.testing.assert_allclose(gt.ravel(), Jm.T @ go.ravel(), atol=1e-13)


def test_hyperparameter_defaults_match_the_paper():
    rows = {}
    with open(os.path.join(GOLDEN, "paper_hyperparameters.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                rows[k] = float(v)
    assert dts_inputs.LAMBDA == rows["lambda"]
    assert dts_inputs.STEP == rows["step"]
    assert dts_inputs.polygon_256()["filter_iters"] == 3
