"""Seeded synthetic inputs for the Domain Transform Solver workloads.

This module is shared by the FP64 oracle side and the GPU side.  It holds none of the
solver's arithmetic: it only draws random scenes with the shapes, value ranges and
structure of the workloads the paper evaluates (Bapat & Frahm, "The Domain Transform
Solver", ECCV 2018):

* guides are colour (or multi-band) images normalised to [0, 1] (Sec. 4, "Stereo
  Optimization" and "Depth super-resolution" paragraphs);
* targets are piecewise-constant or piecewise-planar maps with noise and outliers,
  standing in for an MC-CNN disparity map (Sec. 3.3) or an upsampled low-resolution
  depth map (Sec. 3.5);
* confidences are per-pixel weights c_i >= 0 (Sec. 3.1, Eq. (2)).

The datasets the paper measures on (Middlebury 2014, the Ferstl et al. depth set) are
not used; these scenes stand in for them with the same shapes.  Every array is float32
in planar layout: guide [Cg][H][W], target/confidence [C][H][W].

Randomness comes only from ``numpy.random.default_rng`` seeded with fixed integers or
integer tuples, so every machine produces bit-identical arrays.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "polygon_scene",
    "polygon_256",
    "disparity_1920x1080",
    "multispectral_shape",
    "multispectral_labels",
    "multispectral_guide_band",
    "multispectral_target",
    "multispectral_10240",
    "uneven_batch_64",
    "rgb_batch_8x1024",
    "random_case",
]

# Hyper-parameters shared by every workload: lambda and the gradient-descent step, both
# 0.99 in the paper's experiments (Sec. 4), and three domain-transform filter iterations
# per smoothing step.
LAMBDA = 0.99
STEP = 0.99
FILTER_ITERS = 3


def _convex_polygon_mask(H, W, cx, cy, radius, angles):
    """Mask of the convex polygon whose vertices sit on a circle, inside its bounding box.

    Vertices at sorted angles on a circle are always in convex position; a pixel centre is
    inside when it lies on the left of every edge (counter-clockwise order).
    Returns (y0, y1, x0, x1, inside) with ``inside`` of shape (y1-y0, x1-x0), or None."""
    vx = cx + radius * np.cos(angles)
    vy = cy + radius * np.sin(angles)
    x0 = max(int(np.floor(vx.min())), 0)
    x1 = min(int(np.ceil(vx.max())) + 1, W)
    y0 = max(int(np.floor(vy.min())), 0)
    y1 = min(int(np.ceil(vy.max())) + 1, H)
    if x0 >= x1 or y0 >= y1:
        return None
    px = np.arange(x0, x1, dtype=np.float64)[None, :] + 0.5
    py = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5
    inside = np.ones((y1 - y0, x1 - x0), dtype=bool)
    n = len(angles)
    for i in range(n):
        ax, ay = vx[i], vy[i]
        bx, by = vx[(i + 1) % n], vy[(i + 1) % n]
        inside &= (bx - ax) * (py - ay) - (by - ay) * (px - ax) >= 0.0
    return y0, y1, x0, x1, inside


def polygon_scene(rng, H, W, Cg, n_poly):
    """Piecewise-smooth guide made of ``n_poly`` convex polygons over a flat background.

    Each polygon has 3-8 vertices at sorted random angles on a circle of radius
    U[0.1, 0.35]*min(H, W) around a centre U[0,W) x U[0,H); its colour is U[0,1]^Cg plus a
    per-channel linear ramp with gradient U[-0.3, 0.3] per image width (and height).
    Polygons are painted in order; the label map records the topmost one (0 = background).
    Returns (guide_without_noise float64 [Cg][H][W], labels int32 [H][W])."""
    guide = np.empty((Cg, H, W), dtype=np.float64)
    guide[:] = rng.uniform(0.0, 1.0, size=Cg)[:, None, None]
    labels = np.zeros((H, W), dtype=np.int32)
    xs = (np.arange(W, dtype=np.float64) + 0.5)[None, :]
    ys = (np.arange(H, dtype=np.float64) + 0.5)[:, None]
    for p in range(n_poly):
        nv = int(rng.integers(3, 9))
        angles = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=nv))
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        radius = rng.uniform(0.1, 0.35) * min(H, W)
        base = rng.uniform(0.0, 1.0, size=Cg)
        gx = rng.uniform(-0.3, 0.3, size=Cg)
        gy = rng.uniform(-0.3, 0.3, size=Cg)
        box = _convex_polygon_mask(H, W, cx, cy, radius, angles)
        if box is None:
            continue
        y0, y1, x0, x1, inside = box
        labels[y0:y1, x0:x1][inside] = p + 1
        bx = xs[:, x0:x1] - cx
        by = ys[y0:y1, :] - cy
        for k in range(Cg):
            ramp = base[k] + gx[k] * bx / W + gy[k] * by / H
            sub = guide[k, y0:y1, x0:x1]
            sub[inside] = np.broadcast_to(ramp, inside.shape)[inside]
    return guide, labels


def _noisy_guide(rng, guide, sd):
    g = guide + sd * rng.standard_normal(size=guide.shape, dtype=np.float32)
    return np.clip(g, 0.0, 1.0).astype(np.float32)


def _polygon_case(seed, H, W, Cg, Ct, n_poly):
    """The polygon-scene recipe at any size: polygon guide with noise sd 0.02, per-label
    U[0,1]^Ct target plus noise sd 0.05 clipped to [0,1], confidence U[0.1,1]^Ct."""
    rng = np.random.default_rng(seed)
    clean, labels = polygon_scene(rng, H, W, Cg, n_poly)
    guide = _noisy_guide(rng, clean, 0.02)
    values = rng.uniform(0.0, 1.0, size=(n_poly + 1, Ct))
    target = values[labels].transpose(2, 0, 1) + rng.normal(0.0, 0.05, size=(Ct, H, W))
    target = np.clip(target, 0.0, 1.0).astype(np.float32)
    conf = rng.uniform(0.1, 1.0, size=(Ct, H, W)).astype(np.float32)
    return guide, target, conf, labels


def polygon_256(seed=0):
    """256x256 RGB guide, 12 polygons, 1-channel target; sigma_s=8, sigma_r=0.2, T=10."""
    guide, target, conf, _ = _polygon_case(seed, 256, 256, 3, 1, 12)
    return dict(name="polygon 256x256 RGB->1, T=10", guide=guide, target=target, conf=conf,
                sigma_s=8.0, sigma_r=0.2, filter_iters=FILTER_ITERS, solver_iters=10,
                lam=LAMBDA, step=STEP, value_range=1.0)


def _disparity_parts(seed):
    H, W, Cg, n_poly = 1080, 1920, 3, 32
    rng = np.random.default_rng(seed)
    clean, labels = polygon_scene(rng, H, W, Cg, n_poly)
    guide = _noisy_guide(rng, clean, 0.02)
    a = rng.uniform(16.0, 224.0, size=n_poly + 1)
    b = rng.uniform(-16.0, 16.0, size=n_poly + 1)
    c = rng.uniform(-16.0, 16.0, size=n_poly + 1)
    xs = np.arange(W, dtype=np.float64)[None, :] / W
    ys = np.arange(H, dtype=np.float64)[:, None] / H
    disp = a[labels] + b[labels] * xs + c[labels] * ys
    top = np.nextafter(np.float32(256.0), np.float32(0.0))
    disp = np.clip(disp, 0.0, float(top))
    clean_disp = disp
    outlier = rng.uniform(0.0, 1.0, size=(H, W)) < 0.10
    disp = np.where(outlier, rng.uniform(0.0, 256.0, size=(H, W)), disp)
    disp = np.minimum(disp, float(top))
    conf = np.where(outlier, 0.05, rng.uniform(0.5, 1.0, size=(H, W)))
    return guide, clean_disp, disp, conf


def disparity_1920x1080(seed=1):
    """1920x1080 RGB guide (32 polygons) with a disparity-like target in [0, 256).

    The stereo-refinement stand-in: per-label planar disparity a + b*x/W + c*y/H with
    a ~ U[16,224], b, c ~ U[-16,16], clipped to [0,256); 10% of pixels replaced by
    U[0,256) outliers; confidence 0.05 on outliers and U[0.5,1] elsewhere;
    sigma_s=16, sigma_r=0.1, T=20."""
    guide, _, disp, conf = _disparity_parts(seed)
    return dict(name="disparity 1920x1080 RGB->1, T=20", guide=guide,
                target=disp.astype(np.float32)[None], conf=conf.astype(np.float32)[None],
                sigma_s=16.0, sigma_r=0.1, filter_iters=FILTER_ITERS, solver_iters=20,
                lam=LAMBDA, step=STEP, value_range=256.0)


def warp_right(left, disp):
    """Right image of a synthetic rectified pair: I_R(u, y) = I_L(u + d(u, y), y), read
    linearly along the row and clamped at the borders, so that I_L(x) is close to
    I_R(x - d) wherever d varies slowly.  left [C][H][W], disp [H][W] in pixels."""
    C, H, W = left.shape
    u = np.arange(W, dtype=np.float64)
    out = np.empty_like(left)
    for y in range(H):
        pos = np.clip(u + disp[y], 0.0, W - 1.0)
        for k in range(C):
            out[k, y] = np.interp(pos, u, left[k, y])
    return out.astype(np.float32)


STEREO_GAMMA = 0.001  # Sec. 4, stereo optimisation
STEREO_EPS = 0.001    # Charbonnier epsilon of Sec. 3.3


def stereo_pair_1920x1080(seed=1):
    """The 1920x1080 disparity scene as a stereo pair: the guide is the left image, the right image
    is warped by the clean planar disparity, the target is the disparity with its 10%
    outliers.  gamma and epsilon of the stereo refinement, sigma_s=16, sigma_r=0.1, T=20."""
    guide, clean_disp, disp, conf = _disparity_parts(seed)
    right = warp_right(guide, clean_disp)
    return dict(name="stereo 1920x1080 RGB pair, disparity target, T=20", left=guide, right=right,
                target=disp.astype(np.float32)[None], conf=conf.astype(np.float32)[None],
                sigma_s=16.0, sigma_r=0.1, filter_iters=FILTER_ITERS, solver_iters=20,
                lam=LAMBDA, step=STEP, gamma=STEREO_GAMMA, eps=STEREO_EPS, value_range=256.0)


def stereo_case(seed, H, W, Cg=3, d_max=16.0, sigma_s=8.0, sigma_r=0.2, T=5, gamma=STEREO_GAMMA,
                eps=STEREO_EPS):
    """A small synthetic stereo pair: polygon-scene left image, per-label planar
    disparity in [0, d_max) with 10% outliers, right image warped by the clean disparity."""
    rng = np.random.default_rng(seed)
    n_poly = 8
    clean, labels = polygon_scene(rng, H, W, Cg, n_poly)
    left = _noisy_guide(rng, clean, 0.02)
    a = rng.uniform(0.0, 0.8 * d_max, size=n_poly + 1)
    b = rng.uniform(-0.1 * d_max, 0.1 * d_max, size=n_poly + 1)
    xs = np.arange(W, dtype=np.float64)[None, :] / max(W, 1)
    disp = np.clip(a[labels] + b[labels] * xs, 0.0, d_max)
    outlier = rng.uniform(0.0, 1.0, size=(H, W)) < 0.10
    target = np.where(outlier, rng.uniform(0.0, d_max, size=(H, W)), disp)
    conf = np.where(outlier, 0.05, rng.uniform(0.5, 1.0, size=(H, W)))
    return dict(name=f"stereo {H}x{W} Cg={Cg} seed={seed}", left=left, right=warp_right(left, disp),
                target=target.astype(np.float32)[None], conf=conf.astype(np.float32)[None],
                sigma_s=sigma_s, sigma_r=sigma_r, filter_iters=FILTER_ITERS, solver_iters=T,
                lam=LAMBDA, step=STEP, gamma=gamma, eps=eps, value_range=d_max)


# ---------------------------------------------------------------------------------------
# Multispectral scene: 10240 x 10240, 16 bands.  Generated in row blocks with per-block seeds so any
# horizontal band can be produced on its own and equals the same rows of the full image.
# ---------------------------------------------------------------------------------------
MS_H = 10240
MS_W = 10240
MS_BANDS = 16
MS_BLOCK = 512
MS_SEED = 2


def multispectral_shape():
    return MS_H, MS_W, MS_BANDS


def _ms_fields(seed):
    rng = np.random.default_rng([seed, 0])
    fields = rng.standard_normal((2, 161, 161))
    cuts = [np.quantile(f, [1.0 / 3.0, 2.0 / 3.0]) for f in fields]
    rng1 = np.random.default_rng([seed, 1])
    base = rng1.uniform(0.1, 0.6, size=9)
    gain = rng1.uniform(0.5, 1.5, size=(9, MS_BANDS))
    value = rng1.uniform(0.0, 1.0, size=9)
    return fields, cuts, base, gain, value


def _bilinear_rows(field, ys, W):
    """Bilinear (corner-aligned) upsampling of a 161x161 field to rows ``ys`` of width W."""
    n = field.shape[0] - 1
    fy = ys.astype(np.float64) * n / (MS_H - 1)
    iy = np.minimum(np.floor(fy).astype(np.int64), n - 1)
    ty = (fy - iy)[:, None]
    rows = (1.0 - ty) * field[iy] + ty * field[iy + 1]
    fx = np.arange(W, dtype=np.float64) * n / (W - 1)
    ix = np.minimum(np.floor(fx).astype(np.int64), n - 1)
    tx = (fx - ix)[None, :]
    return (1.0 - tx) * rows[:, ix] + tx * rows[:, ix + 1]


def _ms_region(fields, cuts, ys, W):
    lab = np.zeros((len(ys), W), dtype=np.int32)
    for f, (q1, q2), scale in zip(fields, cuts, (3, 1)):
        up = _bilinear_rows(f, ys, W)
        lab += scale * ((up > q1).astype(np.int32) + (up > q2).astype(np.int32))
    return lab


def multispectral_labels(r0, r1, seed=MS_SEED):
    """Region labels (0..8) of rows [r0, r1): two smooth random fields (161x161 Gaussian
    noise, bilinearly upsampled) thresholded at the terciles of the low-res fields."""
    fields, cuts, *_ = _ms_fields(seed)
    return _ms_region(fields, cuts, np.arange(r0, r1), MS_W)


def multispectral_guide_band(k, r0, r1, labels=None, seed=MS_SEED):
    """Band k of the 16-band guide on rows [r0, r1) (r0, r1 multiples of 512):
    clip(gain[region, k] * base[region] + N(0, 0.01), 0, 1)."""
    fields, cuts, base, gain, _ = _ms_fields(seed)
    if labels is None:
        labels = _ms_region(fields, cuts, np.arange(r0, r1), MS_W)
    lut = (gain[:, k] * base).astype(np.float32)
    out = np.empty((r1 - r0, MS_W), dtype=np.float32)
    for b0 in range(r0, r1, MS_BLOCK):
        b = b0 // MS_BLOCK
        rng = np.random.default_rng([seed, 2, k, b])
        sl = slice(b0 - r0, b0 - r0 + MS_BLOCK)
        noise = rng.standard_normal((MS_BLOCK, MS_W), dtype=np.float32)
        out[sl] = lut[labels[sl]] + np.float32(0.01) * noise
    np.clip(out, 0.0, 1.0, out=out)
    return out


_LOWRES_CACHE = {}


def _ms_lowres_target(seed):
    if seed not in _LOWRES_CACHE:
        fields, cuts, _, _, value = _ms_fields(seed)
        centres = np.arange(8, MS_H, 16)
        low_lab = _ms_region(fields, cuts, centres, MS_W)[:, 8::16]
        _LOWRES_CACHE[seed] = value[low_lab].astype(np.float32)
    return _LOWRES_CACHE[seed]


def multispectral_target(r0, r1, seed=MS_SEED):
    """Target rows [r0, r1): the region value at the centre of each 16x16 block (a 640x640
    low-resolution map), nearest-upsampled x16, plus N(0, 0.02), clipped to [0,1]."""
    low = _ms_lowres_target(seed)
    out = np.empty((r1 - r0, MS_W), dtype=np.float32)
    for b0 in range(r0, r1, MS_BLOCK):
        b = b0 // MS_BLOCK
        rng = np.random.default_rng([seed, 3, b])
        rows = np.arange(b0, b0 + MS_BLOCK) // 16
        up = np.repeat(low[rows], 16, axis=1)
        noise = rng.standard_normal((MS_BLOCK, MS_W), dtype=np.float32)
        out[b0 - r0:b0 - r0 + MS_BLOCK] = up + np.float32(0.02) * noise
    np.clip(out, 0.0, 1.0, out=out)
    return out


def multispectral_10240(rows=(0, MS_H), seed=MS_SEED, workers=8):
    """The 10240x10240, 16-band, 1-channel multispectral workload (or a full-width band
    of it): confidence 1, sigma_s=32, sigma_r=0.15, T=10.  The full guide is 6.7 GB.
    Tiles (band, 512-row block) are independently seeded, so a thread pool fills them in
    any order with identical results."""
    from concurrent.futures import ThreadPoolExecutor

    r0, r1 = rows
    assert r0 % MS_BLOCK == 0 and r1 % MS_BLOCK == 0 and 0 <= r0 < r1 <= MS_H
    guide = np.empty((MS_BANDS, r1 - r0, MS_W), dtype=np.float32)
    blocks = list(range(r0, r1, MS_BLOCK))
    with ThreadPoolExecutor(max(1, workers)) as ex:
        labels = dict(zip(blocks, ex.map(lambda b0: multispectral_labels(b0, b0 + MS_BLOCK, seed),
                                         blocks)))

        def fill(job):
            k, b0 = job
            guide[k, b0 - r0:b0 - r0 + MS_BLOCK] = multispectral_guide_band(
                k, b0, b0 + MS_BLOCK, labels=labels[b0], seed=seed)

        list(ex.map(fill, [(k, b0) for k in range(MS_BANDS) for b0 in blocks]))
        target = np.empty((1, r1 - r0, MS_W), dtype=np.float32)

        def fill_t(b0):
            target[0, b0 - r0:b0 - r0 + MS_BLOCK] = multispectral_target(b0, b0 + MS_BLOCK, seed)

        list(ex.map(fill_t, blocks))
    conf = np.ones_like(target)
    return dict(name="multispectral 10240x10240 16-band->1, T=10", guide=guide, target=target, conf=conf,
                sigma_s=32.0, sigma_r=0.15, filter_iters=FILTER_ITERS, solver_iters=10,
                lam=LAMBDA, step=STEP, value_range=1.0)


def uneven_batch_64(n=64, seed0=100, workers=8):
    """64 uneven instances: W ~ U{320..1920}, H ~ U{240..1080}, Cg in {1,3,8,16},
    Ct in {1,2,3}, sigma_s ~ U[4,32], sigma_r ~ U[0.05,0.3], T=10; polygon scenes.
    Instances are independently seeded, so a thread pool builds them in any order."""
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        rng = np.random.default_rng(seed0 + i)
        W = int(rng.integers(320, 1921))
        H = int(rng.integers(240, 1081))
        Cg = int(rng.choice([1, 3, 8, 16]))
        Ct = int(rng.integers(1, 4))
        sigma_s = float(rng.uniform(4.0, 32.0))
        sigma_r = float(rng.uniform(0.05, 0.3))
        guide, target, conf, _ = _polygon_case(seed0 + 1000 + i, H, W, Cg, Ct, 12)
        return dict(name=f"uneven[{i}] {W}x{H} Cg={Cg} Ct={Ct}", guide=guide, target=target,
                    conf=conf, sigma_s=sigma_s, sigma_r=sigma_r, filter_iters=FILTER_ITERS,
                    solver_iters=10, lam=LAMBDA, step=STEP, value_range=1.0)

    with ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(one, range(n)))


def rgb_batch_8x1024(n=8, size=1024, seed0=200, ref_seed=299, workers=8):
    """Batch of 8 1024x1024 RGB guides with 3-channel targets and confidences (polygon-scene
    scenes), T=15, and the seeded reference r ~ U[0,1] of the loss sum((z^T - r)^2)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max(1, workers)) as ex:
        parts = list(ex.map(lambda i: _polygon_case(seed0 + i, size, size, 3, 3, 12), range(n)))
    rng = np.random.default_rng(ref_seed)
    ref = rng.uniform(0.0, 1.0, size=(n, 3, size, size)).astype(np.float32)
    return dict(name=f"rgb batch {n}x{size}x{size} RGB->3, T=15",
                guide=np.stack([p[0] for p in parts]), target=np.stack([p[1] for p in parts]),
                conf=np.stack([p[2] for p in parts]), ref=ref,
                sigma_s=8.0, sigma_r=0.2, filter_iters=FILTER_ITERS, solver_iters=15,
                lam=LAMBDA, step=STEP, value_range=1.0)


def random_case(seed, H, W, Cg, Ct, Cc=None, sigma_s=6.0, sigma_r=0.25, T=3, n_poly=4):
    """Small polygon-scene case of any shape for parity tests (Cc = 1 or Ct)."""
    Cc = Ct if Cc is None else Cc
    guide, target, conf, _ = _polygon_case(seed, H, W, Cg, Ct, n_poly)
    if Cc == 1:
        conf = conf[:1].copy()
    return dict(name=f"rand{seed} {W}x{H} Cg={Cg} Ct={Ct} Cc={Cc}", guide=guide, target=target,
                conf=conf, sigma_s=sigma_s, sigma_r=sigma_r, filter_iters=FILTER_ITERS,
                solver_iters=T, lam=LAMBDA, step=STEP, value_range=1.0)
