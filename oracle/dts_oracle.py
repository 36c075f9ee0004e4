"""Plain FP64 CPU oracle of the Domain Transform Solver hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  The product path (the HIP library and its
Python binding) never imports, links or calls it, and it shares no code with them.

Source: A. Bapat and J.-M. Frahm, "The Domain Transform Solver", ECCV 2018
(arXiv:1805.04590).  Equations are numbered in order of appearance:
  Eq. (2)  the objective without the application term (Sec. 3.1),
  Eq. (3)  its gradient, the gradient-descent direction (Sec. 3.1),
  Eq. (4)  the per-pixel stationarity condition (Sec. 3.1),
  Eq. (7)  the variance-based confidence (Sec. 3.1),
  Eq. (8)  the local isometry of the domain transform (Sec. 3.2),
  Eq. (9)  the domain transform as an integral of the arc-length element (Sec. 3.2),
  Eq. (10) the edge-aware mean through a kernel H on transformed distances (Sec. 3.2).
The recursive-filter form of the edge-aware mean (feedback coefficient a = exp(-sqrt(2) /
sigma_H), weights a^d, and the halving sigma_H schedule over filter iterations) is the one
of Gastal & Oliveira's domain transform, which Sec. 2 and Sec. 3.2 of the paper build on;
Sec. 3.2 states that the 2-D filter alternates passes along X and then Y.

Readings taken where the paper is silent or garbled (each listed in the design notes):
  R1  the integrand of Eq. (9) is sqrt(1 + (sigma_s/sigma_r)^2 * sum_k I_k'(x)^2), the
      squares following from Eq. (8), discretised with backward differences between
      neighbouring pixels;
  R2  the kernel H of Eq. (10) is the first-order recursive filter with weights a^d;
  R3  a_i = exp(-sqrt(2)/sigma_Hi), sigma_Hi = sigma_s*sqrt(3)*2^(N-i)/sqrt(4^N - 1);
  R4  boundaries: J[0] = f[0] and K[L-1] = J[L-1], no padding;
  R5  every filter iteration runs rows then columns, causal then anticausal; the weight
      w[n] links samples n-1 and n;
  R6  the update follows Eq. (3) as printed: z <- z - step*(lambda*(z - DT(z)) + c*(z - t));
  R8  z^0 = t;  R11 target channels share the guide's distances; confidence has one
      channel (broadcast) or one per target channel;  R12 sigma_x = sigma_y = sigma_s.

Arrays: guide [Cg][H][W], signals [C][H][W]; inputs may be float32, every computation
here is float64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "distances",
    "feedback_coefficients",
    "rf1d_lines",
    "rf1d_lines_adjoint",
    "dt_filter",
    "solve",
    "solve_backward",
    "energy_e2",
    "residual",
    "dense_filter_matrix",
    "variance_confidence",
    "support_lines",
    "support",
    "support_confidence",
    "box_codes",
    "box_radii",
    "box_lines",
    "box_filter",
    "solve_box",
    "sample_row_linear",
    "stereo_data_gradient",
    "energy_stereo",
    "solve_stereo",
]


# ----------------------------------------------------------------------------------------
# O1: transformed distances (Sec. 3.2, Eq. (8)-(9), reading R1)
# ----------------------------------------------------------------------------------------
def distances(guide, sigma_s, sigma_r):
    """Per-pixel arc-length increments of the domain transform along x and along y.

    dx[y, x] = sqrt(1 + s^2 * sum_k (I_k[y, x] - I_k[y, x-1])^2) for x >= 1 and
    dy[y, x] = sqrt(1 + s^2 * sum_k (I_k[y, x] - I_k[y-1, x])^2) for y >= 1, with
    s = sigma_s / sigma_r.  The discrete form of the integrand of Eq. (9): the squared
    step in [x, I] space of Eq. (8), with the range axis scaled by sigma_s/sigma_r.
    Entries dx[:, 0] and dy[0, :] are never used by the filter and are set to 1.

    ``guide`` may be an array [Cg][H][W] or any iterable of [H][W] bands (consumed one
    band at a time, so a very large guide need not be upcast at once)."""
    s2 = (float(sigma_s) / float(sigma_r)) ** 2
    acc_x = None
    acc_y = None
    for band in guide:
        b = np.asarray(band, dtype=np.float64)
        if acc_x is None:
            acc_x = np.zeros_like(b)
            acc_y = np.zeros_like(b)
        acc_x[:, 1:] += (b[:, 1:] - b[:, :-1]) ** 2
        acc_y[1:, :] += (b[1:, :] - b[:-1, :]) ** 2
    dx = np.sqrt(1.0 + s2 * acc_x)
    dy = np.sqrt(1.0 + s2 * acc_y)
    dx[:, 0] = 1.0
    dy[0, :] = 1.0
    return dx, dy


# ----------------------------------------------------------------------------------------
# O2: filter schedule (Gastal & Oliveira's recursive filter; reading R3)
# ----------------------------------------------------------------------------------------
def feedback_coefficients(sigma_s, filter_iters):
    """a_i = exp(-sqrt(2)/sigma_Hi), i = 1..N, with the halving schedule
    sigma_Hi = sigma_s * sqrt(3) * 2^(N-i) / sqrt(4^N - 1), whose squares sum to sigma_s^2."""
    N = int(filter_iters)
    out = []
    for i in range(1, N + 1):
        sigma_h = float(sigma_s) * math.sqrt(3.0) * 2.0 ** (N - i) / math.sqrt(4.0 ** N - 1.0)
        out.append(math.exp(-math.sqrt(2.0) / sigma_h))
    return out


# ----------------------------------------------------------------------------------------
# O3: one 1-D recursive pass, causal then anticausal (readings R4, R5)
# ----------------------------------------------------------------------------------------
def rf1d_lines(f, w, return_intermediates=False):
    """Run the recursive filter along axis 0 of ``f`` (all other axes are independent lines).

    causal:     J[0] = f[0];       J[n] = (1 - w[n]) f[n] + w[n] J[n-1],      n = 1..L-1
    anticausal: K[L-1] = J[L-1];   K[n] = (1 - w[n+1]) J[n] + w[n+1] K[n+1],  n = L-2..0
    ``w`` broadcasts against ``f``; w[0] is never read."""
    f = np.asarray(f, dtype=np.float64)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), f.shape)
    L = f.shape[0]
    J = np.empty_like(f)
    J[0] = f[0]
    for n in range(1, L):
        J[n] = (1.0 - w[n]) * f[n] + w[n] * J[n - 1]
    K = np.empty_like(f)
    K[L - 1] = J[L - 1]
    for n in range(L - 2, -1, -1):
        K[n] = (1.0 - w[n + 1]) * J[n] + w[n + 1] * K[n + 1]
    if return_intermediates:
        return K, J
    return K


def rf1d_lines_adjoint(gK, f, J, K, w):
    """Reverse-mode derivative of ``rf1d_lines`` along axis 0.

    Given dL/dK, returns (dL/df, dL/dw), derived from the two recurrences by the chain rule:
    anticausal adjoint, n = 0..L-1:  rho[n] = gK[n] + w[n] rho[n-1]   (rho[0] = gK[0])
        gJ[n] = (1 - w[n+1]) rho[n] (n <= L-2),  gJ[L-1] = rho[L-1]
        gw[n+1] += rho[n] (K[n+1] - J[n])
    causal adjoint, n = L-1..0:      sig[n] = gJ[n] + w[n+1] sig[n+1]  (sig[L-1] = gJ[L-1])
        gf[n] = (1 - w[n]) sig[n] (n >= 1),  gf[0] = sig[0]
        gw[n] += sig[n] (J[n-1] - f[n])
    ``gw`` has the full shape of ``f`` (not reduced over broadcast axes); gw[0] = 0."""
    gK = np.asarray(gK, dtype=np.float64)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), gK.shape)
    L = gK.shape[0]
    gw = np.zeros_like(gK)
    rho = np.empty_like(gK)
    rho[0] = gK[0]
    for n in range(1, L):
        rho[n] = gK[n] + w[n] * rho[n - 1]
    gJ = np.empty_like(gK)
    gJ[L - 1] = rho[L - 1]
    for n in range(0, L - 1):
        gJ[n] = (1.0 - w[n + 1]) * rho[n]
        gw[n + 1] += rho[n] * (K[n + 1] - J[n])
    sig = np.empty_like(gK)
    sig[L - 1] = gJ[L - 1]
    for n in range(L - 2, -1, -1):
        sig[n] = gJ[n] + w[n + 1] * sig[n + 1]
    gf = np.empty_like(gK)
    gf[0] = sig[0]
    for n in range(1, L):
        gf[n] = (1.0 - w[n]) * sig[n]
        gw[n] += sig[n] * (J[n - 1] - f[n])
    return gf, gw


def _row_pass(sig, wx, keep=False):
    """Filter every row (axis -1) of sig [C][H][W] with weights wx [H][W]."""
    fT = np.ascontiguousarray(np.moveaxis(sig, -1, 0))          # [W][C][H]
    wT = np.ascontiguousarray(wx.T)[:, None, :]                  # [W][1][H]
    out = rf1d_lines(fT, wT, return_intermediates=keep)
    if keep:
        K, J = out
        return np.moveaxis(K, 0, -1).copy(), np.moveaxis(J, 0, -1).copy()
    return np.moveaxis(out, 0, -1).copy()


def _col_pass(sig, wy, keep=False):
    """Filter every column (axis -2) of sig [C][H][W] with weights wy [H][W]."""
    fT = np.ascontiguousarray(np.moveaxis(sig, -2, 0))          # [H][C][W]
    wT = wy[:, None, :]                                          # [H][1][W]
    out = rf1d_lines(fT, wT, return_intermediates=keep)
    if keep:
        K, J = out
        return np.moveaxis(K, 0, -2).copy(), np.moveaxis(J, 0, -2).copy()
    return np.moveaxis(out, 0, -2).copy()


def _pass_weights(dx, dy, sigma_s, filter_iters):
    """Per filter iteration i: (a_i, a_i^dx, a_i^dy)."""
    return [(a, np.power(a, dx), np.power(a, dy))
            for a in feedback_coefficients(sigma_s, filter_iters)]


# ----------------------------------------------------------------------------------------
# O4: the 2-D domain-transform filter, DT(f)  (Sec. 3.2: alternating X then Y passes)
# ----------------------------------------------------------------------------------------
def dt_filter(src, dx, dy, sigma_s, filter_iters):
    """N filter iterations, each a row pass then a column pass, on every channel of
    src [C][H][W] with the same weights."""
    z = np.asarray(src, dtype=np.float64)
    for _, wx, wy in _pass_weights(dx, dy, sigma_s, filter_iters):
        z = _row_pass(z, wx)
        z = _col_pass(z, wy)
    return z


# ----------------------------------------------------------------------------------------
# O5: the solver (Sec. 3.1, Eq. (3); Sec. 4 hyper-parameters; readings R6, R8, R9)
# ----------------------------------------------------------------------------------------
def solve(guide, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10,
          lam=0.99, step=0.99, return_iterates=False, dists=None):
    """Gradient descent on Eq. (2) along the direction of Eq. (3):

        z^0 = t,   z^{k+1} = z^k - step * (lam * (z^k - DT(z^k)) + c * (z^k - t)),

    k = 0..T-1, where DT is the 2-D domain-transform filter guided by ``guide``.
    Returns z^T [Ct][H][W] (and the list z^0..z^T if ``return_iterates``)."""
    t = np.asarray(target, dtype=np.float64)
    c = np.asarray(conf, dtype=np.float64)
    if dists is None:
        dists = distances(guide, sigma_s, sigma_r)
    dx, dy = dists
    z = t.copy()
    iterates = [z.copy()] if return_iterates else None
    for _ in range(int(solver_iters)):
        zbar = dt_filter(z, dx, dy, sigma_s, filter_iters)
        z = z - step * (lam * (z - zbar) + c * (z - t))
        if return_iterates:
            iterates.append(z.copy())
    if return_iterates:
        return z, iterates
    return z


def energy_e2(z, target, conf, dx, dy, sigma_s, filter_iters=3, lam=0.99):
    """E2 = lam/2 * sum (z - DT(z))^2 + 1/2 * sum c (z - t)^2: the energy whose gradient,
    with DT(z) held fixed, is the Eq. (3) direction (reading R6 of Eq. (2)'s data term)."""
    z = np.asarray(z, dtype=np.float64)
    zbar = dt_filter(z, dx, dy, sigma_s, filter_iters)
    t = np.asarray(target, dtype=np.float64)
    c = np.broadcast_to(np.asarray(conf, dtype=np.float64), z.shape)
    return 0.5 * lam * float(np.sum((z - zbar) ** 2)) + 0.5 * float(np.sum(c * (z - t) ** 2))


def residual(z, target, conf, dx, dy, sigma_s, filter_iters=3, lam=0.99):
    """The Eq. (3) gradient lam*(z - DT(z)) + c*(z - t) at z (zero at a stationary point)."""
    z = np.asarray(z, dtype=np.float64)
    zbar = dt_filter(z, dx, dy, sigma_s, filter_iters)
    t = np.asarray(target, dtype=np.float64)
    c = np.asarray(conf, dtype=np.float64)
    return lam * (z - zbar) + c * (z - t)


# ----------------------------------------------------------------------------------------
# O6: adjoint of the whole solve (derived from O1-O5 by the chain rule)
# ----------------------------------------------------------------------------------------
def solve_backward(guide, target, conf, sigma_s, sigma_r, grad_out, filter_iters=3,
                   solver_iters=10, lam=0.99, step=0.99):
    """Gradients of a scalar loss L(z^T) with respect to target, confidence and guide.

    ``grad_out`` = dL/dz^T [Ct][H][W].  The update z^{k+1} = (1 - step*lam - step*c) z^k
    + step*lam*DT(z^k) + step*c*t gives, for k = T-1..0 and g = dL/dz^{k+1}:
        dL/dt += step*c*g,   dL/dc += step*(t - z^k)*g,
        dL/dz^k = (1 - step*lam - step*c)*g + DT^T(step*lam*g),
    where DT^T runs the pass adjoints in reverse pass order and accumulates dL/dw for every
    pass (w = a^d, so dL/dd = dL/dw * w * ln a); finally dL/dt += dL/dz^0 and dL/dd is
    mapped to the guide through the distance formula.  Iterates z^k are recomputed
    forward and the pass intermediates of DT(z^k) are recomputed from z^k.
    Returns (grad_target [Ct][H][W], grad_conf shaped like conf, grad_guide [Cg][H][W])."""
    guide = np.asarray(guide, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    c_in = np.asarray(conf, dtype=np.float64)
    c = np.broadcast_to(c_in, t.shape)
    dx, dy = distances(guide, sigma_s, sigma_r)
    weights = _pass_weights(dx, dy, sigma_s, filter_iters)
    _, iterates = solve(guide, target, conf, sigma_s, sigma_r, filter_iters, solver_iters,
                        lam, step, return_iterates=True, dists=(dx, dy))
    g = np.asarray(grad_out, dtype=np.float64).copy()
    gt = np.zeros_like(t)
    gc = np.zeros_like(t)
    gdx = np.zeros_like(dx)
    gdy = np.zeros_like(dy)
    for k in range(int(solver_iters) - 1, -1, -1):
        zk = iterates[k]
        gt += step * c * g
        gc += step * (t - zk) * g
        # recompute DT(z^k), keeping every pass's input f, causal J and output K
        tape = []
        sig = zk
        for a, wx, wy in weights:
            K, J = _row_pass(sig, wx, keep=True)
            tape.append(("row", a, wx, sig, J, K))
            sig = K
            K, J = _col_pass(sig, wy, keep=True)
            tape.append(("col", a, wy, sig, J, K))
            sig = K
        gsig = step * lam * g
        for kind, a, w, f, J, K in reversed(tape):
            if kind == "row":
                mv = lambda x: np.ascontiguousarray(np.moveaxis(x, -1, 0))  # noqa: E731
                wl = np.ascontiguousarray(w.T)[:, None, :]
                gf, gw = rf1d_lines_adjoint(mv(gsig), mv(f), mv(J), mv(K), wl)
                gf = np.moveaxis(gf, 0, -1)
                gw = np.moveaxis(gw, 0, -1).sum(axis=0)              # sum over channels
                gdx += gw * w * math.log(a)
            else:
                mv = lambda x: np.ascontiguousarray(np.moveaxis(x, -2, 0))  # noqa: E731
                wl = w[:, None, :]
                gf, gw = rf1d_lines_adjoint(mv(gsig), mv(f), mv(J), mv(K), wl)
                gf = np.moveaxis(gf, 0, -2)
                gw = np.moveaxis(gw, 0, -2).sum(axis=0)
                gdy += gw * w * math.log(a)
            gsig = gf
        g = (1.0 - step * lam - step * c) * g + gsig
    gt += g
    # distances -> guide:  d = sqrt(1 + s^2 sum_k D_k^2)  =>  dd/dD_k = s^2 D_k / d
    s2 = (float(sigma_s) / float(sigma_r)) ** 2
    gg = np.zeros_like(guide)
    gdx[:, 0] = 0.0
    gdy[0, :] = 0.0
    for kb in range(guide.shape[0]):
        b = guide[kb]
        Dx = np.zeros_like(b)
        Dx[:, 1:] = b[:, 1:] - b[:, :-1]
        Dy = np.zeros_like(b)
        Dy[1:, :] = b[1:, :] - b[:-1, :]
        ex = gdx * s2 * Dx / dx
        ey = gdy * s2 * Dy / dy
        gg[kb] += ex
        gg[kb][:, :-1] -= ex[:, 1:]
        gg[kb] += ey
        gg[kb][:-1, :] -= ey[1:, :]
    if c_in.shape[0] == 1 and t.shape[0] != 1:
        gc = gc.sum(axis=0, keepdims=True)
    return gt, gc, gg


# ----------------------------------------------------------------------------------------
# Dense form of the filter, for pins on tiny images
# ----------------------------------------------------------------------------------------
def dense_filter_matrix(dx, dy, sigma_s, filter_iters=3):
    """The matrix A with DT(z).ravel() = A @ z.ravel() for one channel, built column by
    column from impulse responses (tiny images only)."""
    H, W = dx.shape
    n = H * W
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros((1, H, W))
        e.flat[j] = 1.0
        A[:, j] = dt_filter(e, dx, dy, sigma_s, filter_iters).ravel()
    return A


# ----------------------------------------------------------------------------------------
# Eq. (7): variance-based confidence (Sec. 3.1), computed from an input before a solve
# ----------------------------------------------------------------------------------------
def variance_confidence(guide, z, sigma_s, sigma_r, sigma_c, filter_iters=3, dists=None):
    """Edge-aware variance of z and the confidence derived from it (Eq. (7)):

        V = DT(z^2) - DT(z)^2,      c = exp(-V / (2 sigma_c^2)),

    where DT is the same domain-transform mean the solver uses (guided by ``guide``),
    read as a local edge-aware estimate of the mean.  z [C][H][W] gives C confidence
    channels.  V is not clipped: rounding can make it slightly negative.
    Returns (c, V)."""
    zz = np.asarray(z, dtype=np.float64)
    if dists is None:
        dists = distances(guide, sigma_s, sigma_r)
    dx, dy = dists
    m1 = dt_filter(zz, dx, dy, sigma_s, filter_iters)
    m2 = dt_filter(zz * zz, dx, dy, sigma_s, filter_iters)
    V = m2 - m1 * m1
    return np.exp(-V / (2.0 * float(sigma_c) ** 2)), V


# ----------------------------------------------------------------------------------------
# Support-weighted confidence (Sec. 3.1, the comparison with the bilateral solver after
# Eq. (6)): the confidence of the gradient-descent update is divided by the support
# sum_j W_ij of the edge-aware kernel, as in the bilateral solver's per-pixel solution.
# Reading R10 (listed in the design notes):
#   - W is the unnormalised form of the 2-D domain-transform kernel: each 1-D pass sums
#     products of the weights a^d along the line on both sides of a pixel, the pixel itself
#     once; the passes alternate rows and columns over the N filter iterations as in O4;
#   - the support is reported relative to that of a pixel deep inside a flat region
#     (every d = 1), whose 1-D pass sum is (1 + a_i) / (1 - a_i): each pass is scaled by
#     (1 - a_i) / (1 + a_i), so the relative support s lies in (0, 1] and is 1 far from
#     edges and borders;
#   - the weighted confidence is c / s: a pixel with less support (near an edge or a
#     border) leans more on its target, one with full support keeps c.
# ----------------------------------------------------------------------------------------
def support_lines(x, w):
    """Two-sided unnormalised recursive sum along axis 0 of ``x``:

        S[n] = sum_j (prod of w[k] over the links k between n and j) x[j],

    evaluated as causal y[n] = x[n] + w[n] y[n-1] (y[0] = x[0]), anticausal
    v[n] = x[n] + w[n+1] v[n+1] (v[L-1] = x[L-1]), S = y + v - x (x[n] counted once).
    ``w`` broadcasts against ``x``; w[0] is never read."""
    x = np.asarray(x, dtype=np.float64)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), x.shape)
    L = x.shape[0]
    y = np.empty_like(x)
    y[0] = x[0]
    for n in range(1, L):
        y[n] = x[n] + w[n] * y[n - 1]
    v = np.empty_like(x)
    v[L - 1] = x[L - 1]
    for n in range(L - 2, -1, -1):
        v[n] = x[n] + w[n + 1] * v[n + 1]
    return y + v - x


def support(guide, sigma_s, sigma_r, filter_iters=3, dists=None):
    """Relative support s [H][W] of the edge-aware kernel (reading R10): the unnormalised
    2-D kernel applied to ones, each 1-D pass scaled by (1 - a_i) / (1 + a_i)."""
    if dists is None:
        dists = distances(guide, sigma_s, sigma_r)
    dx, dy = dists
    s = np.ones(dx.shape, dtype=np.float64)
    for a, wx, wy in _pass_weights(dx, dy, sigma_s, filter_iters):
        m = (1.0 - a) / (1.0 + a)
        s = m * support_lines(s.T, wx.T).T      # rows: lines along x
        s = m * support_lines(s, wy)            # columns: lines along y
    return s


def support_confidence(guide, conf, sigma_s, sigma_r, filter_iters=3, dists=None):
    """Confidence weighted by the inverse relative support, c / s (reading R10);
    conf [Cc][H][W].  Returns (c / s, s)."""
    s = support(guide, sigma_s, sigma_r, filter_iters, dists)
    return np.asarray(conf, dtype=np.float64) / s[None], s


# ----------------------------------------------------------------------------------------
# Box form of the edge-aware mean (Sec. 3.2, Eq. (10) read literally): the kernel H is the
# indicator of |DT_i - DT_j| <= r, i.e. the mean over the pixels of the same line whose
# transformed coordinates lie within r of pixel i's (a normalised convolution).
# Readings (listed in the design notes):
#   B1  the transformed coordinate of a line is the running sum of the arc-length
#       increments d of Eq. (9) (reading R1), ct[0] = 0, ct[n] = ct[n-1] + d[n];
#   B2  the radius, never given, is that of the box with the variance of the recursive
#       form's iteration: r_i = sqrt(3) sigma_Hi, with the same sigma_Hi schedule (R3);
#   B3  iterations alternate rows then columns as in O4;
#   B4  membership is an integer decision: each d is computed in float32 as
#       sqrt(1 + s2 * sum_k (I_k[n] - I_k[n-1])^2) (each operation rounded to nearest,
#       bands summed in order, s2 = the double product (sigma_s/sigma_r)(sigma_s/sigma_r)
#       rounded to float32, sigma_s and sigma_r taken as float32) and coded as
#       q = rint(256 d), the coordinate is the integer sum of the codes, the radius is
#       R_i = floor(256 r_i), and j belongs to i's box iff |ct_i - ct_j| <= R_i.
# ----------------------------------------------------------------------------------------
def box_codes(guide, sigma_s, sigma_r):
    """Integer codes (qx, qy) [H][W] of the arc-length increments in units of 1/256
    pixel (reading B4); qx[:, 0] and qy[0, :] are unused and set to 0."""
    ratio = float(np.float32(sigma_s)) / float(np.float32(sigma_r))
    s2 = np.float32(ratio * ratio)
    acc_x = acc_y = None
    for band in guide:
        b = np.asarray(band, dtype=np.float32)
        if acc_x is None:
            acc_x = np.zeros_like(b)
            acc_y = np.zeros_like(b)
        ex = b[:, 1:] - b[:, :-1]
        ey = b[1:, :] - b[:-1, :]
        acc_x[:, 1:] = acc_x[:, 1:] + ex * ex
        acc_y[1:, :] = acc_y[1:, :] + ey * ey
    one, scale = np.float32(1.0), np.float32(256.0)
    qx = np.rint(np.sqrt(one + s2 * acc_x) * scale).astype(np.int64)
    qy = np.rint(np.sqrt(one + s2 * acc_y) * scale).astype(np.int64)
    qx[:, 0] = 0
    qy[0, :] = 0
    return qx, qy


def box_radii(sigma_s, filter_iters):
    """R_i = floor(256 sqrt(3) sigma_Hi), i = 1..N (readings B2, B4)."""
    N = int(filter_iters)
    out = []
    for i in range(1, N + 1):
        sigma_h = float(np.float32(sigma_s)) * math.sqrt(3.0) * 2.0 ** (N - i) / math.sqrt(4.0 ** N - 1.0)
        out.append(int(math.floor(sigma_h * math.sqrt(3.0) * 256.0)))
    return out


def box_lines(f, q, R):
    """Box mean along axis 0 of ``f`` [L][M] (columns are independent lines) with codes
    q [L][M]: out[n] = mean of f[j] over the j with |ct[n] - ct[j]| <= R."""
    f = np.asarray(f, dtype=np.float64)
    q = np.asarray(q, dtype=np.int64).copy()
    q[0] = 0
    ct = np.cumsum(q, axis=0)
    out = np.empty_like(f)
    for m in range(f.shape[1]):
        c = ct[:, m]
        lo = np.searchsorted(c, c - R, side="left")          # first j with ct[j] >= ct[n] - R
        hi = np.searchsorted(c, c + R, side="right") - 1     # last j with ct[j] <= ct[n] + R
        P = np.concatenate([[0.0], np.cumsum(f[:, m])])
        out[:, m] = (P[hi + 1] - P[lo]) / (hi - lo + 1)
    return out


def box_filter(src, qx, qy, sigma_s, filter_iters):
    """N box iterations, each along rows then along columns, on every channel of
    src [C][H][W] with the same codes (readings B1-B4)."""
    z = np.asarray(src, dtype=np.float64)
    out = np.empty_like(z)
    for R in box_radii(sigma_s, filter_iters):
        for c in range(z.shape[0]):
            out[c] = box_lines(z[c].T, qx.T, R).T
            out[c] = box_lines(out[c], qy, R)
        z = out.copy()
    return z


def solve_box(guide, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10,
              lam=0.99, step=0.99):
    """The solver of O5 with the box form of the edge-aware mean:
    z^0 = t, z^{k+1} = z^k - step (lam (z^k - BOX(z^k)) + c (z^k - t))."""
    qx, qy = box_codes(guide, sigma_s, sigma_r)
    t = np.asarray(target, dtype=np.float64)
    c = np.asarray(conf, dtype=np.float64)
    z = t.copy()
    for _ in range(int(solver_iters)):
        zbar = box_filter(z, qx, qy, sigma_s, filter_iters)
        z = z - step * (lam * (z - zbar) + c * (z - t))
    return z


# ----------------------------------------------------------------------------------------
# Stereo (Sec. 3.3, Eq. (11)): edge-aware smoothness, Charbonnier target term, and the
# photometric term of a rectified pair.  Readings (listed in the design notes):
#   S1  disparities are in pixels: the left pixel (x, y) matches the right image at
#       (x - z, y) on the same row;
#   S2  the right image is sampled linearly along x, the sample position clamped to
#       [0, W - 1]; the derivative is the slope of the segment the sample falls in
#       (segment [x0, x0 + 1] with x0 = min(floor(x_s), W - 2)), and 0 where the position
#       was clamped (the sample does not move there); a one-pixel-wide image has slope 0;
#   S3  colour images: the photometric term sums the squared differences over channels;
#   S4  the update is gradient descent on Eq. (11) with the edge-aware mean held fixed,
#       as Eq. (3) is for Eq. (2):  z <- z - step * (lam (z - DT(z)) + D(z)),
#       D = c rho'(z - t) + gamma sum_k (I_L,k - I_R,k(x - z)) dI_R,k/dx(x - z),
#       rho(r) = sqrt(r^2 + eps^2) (so rho'(r) = r / sqrt(r^2 + eps^2));
#   S5  the left image is the guide of the edge-aware mean.
# ----------------------------------------------------------------------------------------
def sample_row_linear(img, xs):
    """Linear interpolation of img [C][H][W] along x at positions xs [H][W] (same row),
    clamped to [0, W - 1] (reading S2).  Returns (values, slopes), both [C][H][W]; the
    slope is 0 where the position was clamped."""
    I = np.asarray(img, dtype=np.float64)
    C, H, W = I.shape
    xr = np.asarray(xs, dtype=np.float64)
    x = np.clip(xr, 0.0, W - 1.0)
    if W == 1:
        return np.broadcast_to(I, (C, H, W)).copy(), np.zeros((C, H, W))
    x0 = np.minimum(np.floor(x), W - 2).astype(np.int64)
    fr = x - x0
    rows = np.arange(H)[:, None]
    left = I[:, rows, x0]
    right = I[:, rows, x0 + 1]
    inside = (xr >= 0.0) & (xr <= W - 1.0)
    return left + fr * (right - left), np.where(inside, right - left, 0.0)


def stereo_data_gradient(left, right, z, target, conf, gamma, eps):
    """D(z) of reading S4: the Charbonnier target term's derivative plus the photometric
    term's derivative with respect to the disparity, per pixel ([1][H][W])."""
    zz = np.asarray(z, dtype=np.float64)[0]
    t = np.asarray(target, dtype=np.float64)[0]
    c = np.asarray(conf, dtype=np.float64)[0]
    IL = np.asarray(left, dtype=np.float64)
    H, W = zz.shape
    xs = np.arange(W)[None, :] - zz
    val, slope = sample_row_linear(right, xs)
    r = zz - t
    photo = gamma * np.sum((IL - val) * slope, axis=0)
    return (c * r / np.sqrt(r * r + eps * eps) + photo)[None]


def energy_stereo(z, zbar, left, right, target, conf, lam, gamma, eps):
    """Eq. (11) with the Charbonnier target term (reading S4), for a given mean zbar."""
    zz = np.asarray(z, dtype=np.float64)[0]
    t = np.asarray(target, dtype=np.float64)[0]
    c = np.asarray(conf, dtype=np.float64)[0]
    W = zz.shape[1]
    val, _ = sample_row_linear(right, np.arange(W)[None, :] - zz)
    photo = 0.5 * gamma * np.sum((np.asarray(left, dtype=np.float64) - val) ** 2)
    return (0.5 * lam * float(np.sum((zz - np.asarray(zbar, dtype=np.float64)[0]) ** 2))
            + float(np.sum(c * np.sqrt((zz - t) ** 2 + eps * eps))) + photo)


def solve_stereo(left, right, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10,
                 lam=0.99, step=0.99, gamma=0.001, eps=0.001, return_iterates=False):
    """Stereo refinement (Sec. 3.3, Eq. (11), readings S1-S5): z^0 = t, then
        z^{k+1} = z^k - step * (lam * (z^k - DT(z^k)) + D(z^k)),
    DT guided by the left image.  target and conf are [1][H][W]; returns z^T (and the
    list z^0..z^T if ``return_iterates``)."""
    t = np.asarray(target, dtype=np.float64)
    dx, dy = distances(left, sigma_s, sigma_r)
    z = t.copy()
    iterates = [z.copy()] if return_iterates else None
    for _ in range(int(solver_iters)):
        zbar = dt_filter(z, dx, dy, sigma_s, filter_iters)
        z = z - step * (lam * (z - zbar) + stereo_data_gradient(left, right, z, target, conf, gamma, eps))
        if return_iterates:
            iterates.append(z.copy())
    if return_iterates:
        return z, iterates
    return z

